// adjoint_kernels.hip -- reverse mode of one step x -> x + Delta(F(x); k, gamma)
// with the neighbour sets, threshold masks and clamp states of the forward
// step held fixed.  For a pair in contact with e = x_i - x_j, d = |e|,
// phi(e) = g(d) e with g(d) = f(S - d) / d:
//   A_ij = d phi / d e = g I + g'(d) e e^T / d,  g' = -(f'(delta) d + f) / d^2,
//   f'(delta) = k - gamma rho / (2 sqrt(rho delta)).
// Per step: w_i = (dDelta_i/dF_i)^T lambda_i (mu I, or delta_max/|F| (I - F^ F^T)
// when clamped, or 0 below the threshold), then
//   lambda_m <- lambda_m + sum_{j in contact with m} A_mj (w_m - w_j),
//   dL/dk += sum_i w_i . sum_j delta_ij u_ij,  dL/dgamma -= sum_i w_i . sum_j sqrt(rho delta) u_ij.
//
// The grids of the reverse steps are full builds: the agent of canonical slot
// t sits in loose slot n + t, with storage index perm[t].
#include "force_loop.h"

namespace abm {

constexpr int kAdjThreads = 256;
constexpr int kAdjChunk = 4;   // candidates the walk of the reverse step tests together

int adj_blocks(uint32_t n) { return int((n + kAdjThreads - 1) / kAdjThreads); }

template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_w(Buffers<T> b, int cur, const double* __restrict__ lam,
                                                        double* __restrict__ w) {
    __shared__ double s_k[kAdjThreads], s_g[kAdjThreads];
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    double gk = 0.0, gg = 0.0;
    const uint32_t i = t < b.n ? b.perm[t] : 0xFFFFFFFFu;
    if (t < b.n && i >= b.n) raise_error(b.g, kErrInternal);
    if (i < b.n) {
        const SimGrid& G = b.sims[sim_index(b, t)];
        const V4<T> p = gpos_ptr(b)[b.n + t];
        uint32_t q[3];
        double wi[3] = {0.0, 0.0, 0.0};
        if (G.valid && box_of<T>(G, p, q)) {
            const Pieces P = load_pieces(b, G, q, b.g->stamp, L);
            ForceSum acc;
            force_of<kAdjChunk, T, true>(b, G, p, P, L, acc);
            const Move m = displacement(G, acc.fx, acc.fy, acc.fz);
            if (m.moves) {
                const double li[3] = {lam[3 * size_t(i)], lam[3 * size_t(i) + 1], lam[3 * size_t(i) + 2]};
                if (m.clamped) {
                    const double Fn = m.fnorm;
                    const double fh[3] = {acc.fx / Fn, acc.fy / Fn, acc.fz / Fn};
                    const double dot = li[0] * fh[0] + li[1] * fh[1] + li[2] * fh[2];
                    for (int a = 0; a < 3; ++a) wi[a] = G.delta_max / Fn * (li[a] - dot * fh[a]);
                } else {
                    for (int a = 0; a < 3; ++a) wi[a] = G.mu * li[a];
                }
                gk = wi[0] * acc.kx + wi[1] * acc.ky + wi[2] * acc.kz;
                gg = wi[0] * acc.gx + wi[1] * acc.gy + wi[2] * acc.gz;
            }
        } else {
            raise_error(b.g, kErrInternal);
        }
        for (int a = 0; a < 3; ++a) w[3 * size_t(i) + a] = wi[a];
    }
    // fixed-shape tree reduction: the result does not depend on timing
    s_k[threadIdx.x] = gk;
    s_g[threadIdx.x] = gg;
    __syncthreads();
    for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            s_k[threadIdx.x] += s_k[threadIdx.x + h];
            s_g[threadIdx.x] += s_g[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && blockIdx.x < b.partial_cap) {
        b.partials[2 * blockIdx.x] = s_k[0];
        b.partials[2 * blockIdx.x + 1] = s_g[0];
    }
}

template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_gather(Buffers<T> b, int cur, const double* __restrict__ lam,
                                                             const double* __restrict__ w,
                                                             double* __restrict__ lam_out) {
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.n) return;
    const SimGrid& G = b.sims[sim_index(b, t)];
    const uint32_t m = b.perm[t];
    if (m >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const V4<T>* __restrict__ sp = gpos_ptr(b);
    const V4<T> p = sp[b.n + t];
    uint32_t q[3];
    double acc[3] = {lam[3 * size_t(m)], lam[3 * size_t(m) + 1], lam[3 * size_t(m) + 2]};
    if (G.valid && box_of<T>(G, p, q)) {
        const Pieces P = load_pieces(b, G, q, b.g->stamp, L);
        const double xm = double(p.x), ym = double(p.y), zm = double(p.z);
        const double rm = 0.5 * fabs(double(p.w));
        const double wm[3] = {w[3 * size_t(m)], w[3 * size_t(m) + 1], w[3 * size_t(m) + 2]};
        stream_pieces(L, P, [&](uint32_t u) {
            if (u == b.n + t || u < b.n) return true;
            const uint32_t j = b.perm[u - b.n];
            if (j >= b.n) return true;
            const V4<T> pj = sp[u];
            const double ev3[3] = {xm - double(pj.x), ym - double(pj.y), zm - double(pj.z)};
            const double s2 = (ev3[0] * ev3[0] + ev3[1] * ev3[1]) + ev3[2] * ev3[2];
            if (!(s2 < G.r2)) return true;
            const double rj = 0.5 * fabs(double(pj.w)), S = rm + rj;
            if (!(s2 > 0.0) || !(s2 < S * S)) return true;
            const double dist = sqrt(s2);
            const double delta = S - dist, rho = (rm * rj) / S;
            const double f = G.k * delta - G.gamma * sqrt(rho * delta);
            const double fp = G.k - G.gamma * rho / (2.0 * sqrt(rho * delta));
            const double gd = f / dist;
            const double gprime = -(fp * dist + f) / (dist * dist);
            const double v[3] = {wm[0] - w[3 * size_t(j)], wm[1] - w[3 * size_t(j) + 1], wm[2] - w[3 * size_t(j) + 2]};
            const double ev = ev3[0] * v[0] + ev3[1] * v[1] + ev3[2] * v[2];
            for (int a = 0; a < 3; ++a) acc[a] += gd * v[a] + gprime / dist * ev3[a] * ev;
            return true;
        });
    } else {
        raise_error(b.g, kErrInternal);
    }
    for (int a = 0; a < 3; ++a) lam_out[3 * size_t(m) + a] = acc[a];
}

// dparams[0..1] += the block partials, summed in block order by one block.
__global__ __launch_bounds__(kAdjThreads) void k_adj_finish(const double* __restrict__ partials, int nblocks,
                                                             double* dparams) {
    __shared__ double s_k[kAdjThreads], s_g[kAdjThreads];
    double k = 0.0, g = 0.0;
    for (int i = int(threadIdx.x); i < nblocks; i += kAdjThreads) {
        k += partials[2 * i];
        g += partials[2 * i + 1];
    }
    s_k[threadIdx.x] = k;
    s_g[threadIdx.x] = g;
    __syncthreads();
    for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            s_k[threadIdx.x] += s_k[threadIdx.x + h];
            s_g[threadIdx.x] += s_g[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dparams[0] += s_k[0];
        dparams[1] += s_g[0];
    }
}

// Storage-indexed <-> id-indexed copies of n x 3 double arrays (the adjoint
// keeps lambda and w by storage slot; callers see them by agent id).
__global__ void k_permute3(const uint32_t* __restrict__ ids, uint32_t n, const double* __restrict__ in,
                           double* __restrict__ out, int to_id) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = ids[i];
    if (id >= n) return;
    for (int a = 0; a < 3; ++a) {
        if (to_id)
            out[3 * size_t(id) + a] = in[3 * size_t(i) + a];
        else
            out[3 * size_t(i) + a] = in[3 * size_t(id) + a];
    }
}

void launch_permute3(const uint32_t* ids, uint32_t n, const double* in, double* out, bool to_id, hipStream_t s) {
    hipLaunchKernelGGL(k_permute3, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, in, out, to_id ? 1 : 0);
}

template <class T>
void launch_adj_w(const Buffers<T>& b, int pos_cur, const double* lam, double* w, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_w<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), walk_lds_bytes(kAdjThreads), s, b, pos_cur,
                       lam, w);
}

template <class T>
void launch_adj_gather(const Buffers<T>& b, int pos_cur, const double* lam, const double* w, double* lam_out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adj_gather<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), walk_lds_bytes(kAdjThreads), s, b,
                       pos_cur, lam, w, lam_out);
}

template <class T>
void launch_adj_finish(const Buffers<T>& b, int nblocks, double* dparams, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_finish, dim3(1), dim3(kAdjThreads), 0, s, b.partials, nblocks, dparams);
}

#define ABM_INSTANTIATE(T)                                                                              \
    template void launch_adj_w<T>(const Buffers<T>&, int, const double*, double*, hipStream_t);       \
    template void launch_adj_gather<T>(const Buffers<T>&, int, const double*, const double*, double*, \
                                       hipStream_t);                                                  \
    template void launch_adj_finish<T>(const Buffers<T>&, int, double*, hipStream_t);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
