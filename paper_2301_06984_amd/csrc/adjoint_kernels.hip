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
// t sits in loose slot n + t, with storage index perm[t].  lambda is kept
// by agent id (a re-layout moves agents between storage slots from one
// forward step to the next); w by canonical slot of the step.  A reverse step
// either walks such a grid (k_adj_w, k_adj_gather) or reads the step's
// contact tape, written by k_adj_tape while the forward step had its grid
// (k_adj_tape_w, k_adj_tape_gather): the same contacts in the same order, so
// both give the same sums, bit for bit.
#include "force_loop.h"

namespace abm {

constexpr int kAdjThreads = 256;
constexpr int kAdjChunk = 4;   // candidates the walk of the reverse step tests together

int adj_blocks(uint32_t n) { return int((n + kAdjThreads - 1) / kAdjThreads); }

// w_i = D_i^T lambda_i for agent i (id) with force sums acc, and its terms
// of dL/dk and dL/dgamma.
__device__ __forceinline__ void adjoint_w(const SimGrid& G, const ForceSum& acc, const double* __restrict__ lam,
                                          uint32_t i, double wi[3], double& gk, double& gg) {
    const Move m = displacement(G, acc.fx, acc.fy, acc.fz);
    if (!m.moves) return;
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

// The block's partial sums of dL/dk and dL/dgamma, by a fixed-shape tree (the
// result does not depend on timing); every thread of the block calls it.
__device__ __forceinline__ void block_partials(double* __restrict__ partials, uint32_t cap, double gk, double gg) {
    __shared__ double s_k[kAdjThreads], s_g[kAdjThreads];
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
    if (threadIdx.x == 0 && blockIdx.x < cap) {
        partials[2 * blockIdx.x] = s_k[0];
        partials[2 * blockIdx.x + 1] = s_g[0];
    }
}

template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_w(Buffers<T> b, int ids_cur, const double* __restrict__ lam,
                                                        double* __restrict__ w) {
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    double gk = 0.0, gg = 0.0;
    const uint32_t si = t < b.n ? b.perm[t] : 0xFFFFFFFFu;
    const uint32_t i = si < b.n ? b.ids[ids_cur][si] : 0xFFFFFFFFu;   // the agent's id
    if (t < b.n && i >= b.n) raise_error(b.g, kErrInternal);
    if (i < b.n) {
        const SimGrid& G = b.sims[sim_index(b, t)];
        const V4<T> p = gpos_ptr(b)[b.n + t];
        uint32_t q[3];
        double wi[3] = {0.0, 0.0, 0.0};
        if (G.valid && box_of<T>(G, p, q)) {
            const Pieces P = load_pieces(b, G, q, G.stamp, L);
            ForceSum acc;
            force_of<kAdjChunk, T, true>(b, G, p, P, L, acc);
            adjoint_w(G, acc, lam, i, wi, gk, gg);
        } else {
            raise_error(b.g, kErrInternal);
        }
        for (int a = 0; a < 3; ++a) w[3 * size_t(t) + a] = wi[a];   // by canonical slot: the gather reads it there
    }
    block_partials(b.partials, b.partial_cap, gk, gg);
}

// One term of the update of lambda_m for its contact at loose slot u:
// A_mj (w_m - w_j), zero for a slot that holds no agent.  w is indexed by
// canonical slot (the agent at loose slot n + t has w[t]).
template <class T>
__device__ __forceinline__ void gather_term(const Buffers<T>& b, const SimGrid& G, double xm, double ym, double zm,
                                            double rm, const double wm[3], const double* __restrict__ w,
                                            const V4<T>& pj, uint32_t u, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    if (u < b.n) return;
    const uint32_t j = u - b.n;   // w is kept by canonical slot
    if (j >= b.n) return;
    const double ev3[3] = {xm - double(pj.x), ym - double(pj.y), zm - double(pj.z)};
    const double s2 = (ev3[0] * ev3[0] + ev3[1] * ev3[1]) + ev3[2] * ev3[2];
    const double rj = 0.5 * fabs(double(pj.w)), S = rm + rj;
    const double dist = sqrt(s2);
    const double delta = S - dist, rho = (rm * rj) / S;
    const double f = G.k * delta - G.gamma * sqrt(rho * delta);
    const double fp = G.k - G.gamma * rho / (2.0 * sqrt(rho * delta));
    const double gd = f / dist;
    const double gprime = -(fp * dist + f) / (dist * dist);
    const double v[3] = {wm[0] - w[3 * size_t(j)], wm[1] - w[3 * size_t(j) + 1], wm[2] - w[3 * size_t(j) + 2]};
    const double ev = ev3[0] * v[0] + ev3[1] * v[1] + ev3[2] * v[2];
    for (int a = 0; a < 3; ++a) out[a] = gd * v[a] + gprime / dist * ev3[a] * ev;
}

// lambda_m <- lambda_m + sum_j A_mj (w_m - w_j) over the contacts of m, in
// slot order.  Every lane of the wave takes part (none returns early): the
// contacts, several per agent and uneven, are dealt out over the wave, one
// per lane, and each term goes back to its agent's lane by register
// shuffles; a lane whose queue fills with contacts mid-walk adds those
// itself.  The sums are in slot order either way.
template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_gather(Buffers<T> b, int ids_cur, const double* __restrict__ lam,
                                                             const double* __restrict__ w,
                                                             double* __restrict__ lam_out) {
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, tid = threadIdx.x, bs = blockDim.x;
    const SimGrid& G = b.sims[0];   // the adjoint covers one simulation
    const V4<T>* __restrict__ sp = gpos_ptr(b);
    const uint32_t last = 2u * b.n - 1u;
    uint32_t m = 0xFFFFFFFFu;
    if (t < b.n) {
        const uint32_t si = b.perm[t];
        m = si < b.n ? b.ids[ids_cur][si] : 0xFFFFFFFFu;   // the agent's id
        if (m >= b.n) raise_error(b.g, kErrInternal);
    }
    const bool has = m < b.n;
    V4<T> p{};
    Pieces P;
    double acc[3] = {0.0, 0.0, 0.0}, wm[3] = {0.0, 0.0, 0.0};
    if (has) {
        p = sp[b.n + t];
        for (int a = 0; a < 3; ++a) {
            acc[a] = lam[3 * size_t(m) + a];
            wm[a] = w[3 * size_t(t) + a];
        }
        uint32_t q[3];
        if (G.valid && box_of<T>(G, p, q))
            P = load_pieces(b, G, q, G.stamp, L);
        else
            raise_error(b.g, kErrInternal);
    }
    const double xm = double(p.x), ym = double(p.y), zm = double(p.z);
    const double rm = 0.5 * fabs(double(p.w));
    const uint32_t kept = queue_contacts<kAdjChunk, T>(b, G, p, P, L, [&](uint32_t k) {
        for (uint32_t r = 0; r < k; ++r) {
            const uint32_t u = L.queue[r * bs + tid];
            double o[3];
            gather_term<T>(b, G, xm, ym, zm, rm, wm, w, sp[min(u, last)], u, o);
            for (int a = 0; a < 3; ++a) acc[a] += o[a];
        }
    });
    // the wave's remaining contacts: lane l's rows [0, kept) are pairs
    // [off, off + kept) of the wave, pair x evaluated by lane x mod 64
    const uint32_t lane = uint32_t(lane_id()), wbase = tid - lane;
    uint32_t incl = kept;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= uint32_t(d)) incl += y;
    }
    const uint32_t off = incl - kept, total = __shfl(incl, 63, 64);
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t x = base + lane;
        uint32_t o = 0;   // the pair's agent: the last lane whose pairs start at or before x
        for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint32_t v = __shfl(off, int(o + step), 64);
            o = v <= x ? o + step : o;
        }
        const uint32_t row = x - __shfl(off, int(o), 64);
        const double oxm = __shfl(xm, int(o), 64), oym = __shfl(ym, int(o), 64), ozm = __shfl(zm, int(o), 64);
        const double orm = __shfl(rm, int(o), 64);
        const double owm[3] = {__shfl(wm[0], int(o), 64), __shfl(wm[1], int(o), 64), __shfl(wm[2], int(o), 64)};
        double term[3] = {0.0, 0.0, 0.0};
        if (x < total) {
            const uint32_t u = L.queue[min(row, uint32_t(queue_cap<kAdjChunk>() - 1)) * bs + wbase + o];
            gather_term<T>(b, G, oxm, oym, ozm, orm, owm, w, sp[min(u, last)], u, term);
        }
        // the terms go back to their agent's lane: the j-th of every lane at once
        const uint32_t j0 = max(off, base), j1 = min(off + kept, base + 64u);
        const uint32_t cnt = j1 > j0 ? j1 - j0 : 0u;
        uint32_t most = cnt;
        for (int d = 32; d >= 1; d >>= 1) most = max(most, uint32_t(__shfl_xor(int(most), d, 64)));
        for (uint32_t j = 0; j < most; ++j) {
            const int src = int(min(j0 + j - base, 63u));
            const double v0 = __shfl(term[0], src, 64), v1 = __shfl(term[1], src, 64), v2 = __shfl(term[2], src, 64);
            if (j < cnt) {
                acc[0] += v0;
                acc[1] += v1;
                acc[2] += v2;
            }
        }
    }
    if (has)
        for (int a = 0; a < 3; ++a) lam_out[3 * size_t(m) + a] = acc[a];
}

// ---------------------------------------------------------------- contact tape
// The contacts of every agent on the step's grid (a full build), found by the
// walk of the gather, in the order the force sums them: canonical slot t
// keeps its position, id and contacts' canonical slots (see
// TapeStep).  A count above kTapeWidth is still counted (and raises *worst
// past it), its excess rows are not kept.
template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_tape(Buffers<T> b, int ids_cur, TapeStep tp) {
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, tid = threadIdx.x, bs = blockDim.x, n = b.n;
    const SimGrid& G = b.sims[0];   // the adjoint covers one simulation
    uint32_t i = 0xFFFFFFFFu;
    if (t < n) {
        i = b.perm[t];
        // a full build holds every agent in the append slots [n, 2n)
        if (i >= n || b.g->inc) raise_error(b.g, kErrInternal);
    }
    const bool has = i < n && !b.g->inc;
    V4<T> p{};
    Pieces P;
    if (has) {
        p = gpos_ptr(b)[n + t];
        uint32_t q[3];
        if (G.valid && box_of<T>(G, p, q))
            P = load_pieces(b, G, q, G.stamp, L);
        else
            raise_error(b.g, kErrInternal);
    }
    uint32_t cnt = 0;
    auto emit = [&](uint32_t k) {
        for (uint32_t r = 0; r < k; ++r) {
            const uint32_t u = L.queue[r * bs + tid];
            if (u < n) {
                raise_error(b.g, kErrInternal);
                continue;
            }
            if (cnt < kTapeWidth) tp.list[size_t(cnt) * n + t] = u - n;
            ++cnt;
        }
    };
    emit(queue_contacts<kAdjChunk, T>(b, G, p, P, L, emit));
    if (has) {
        tp.cnt[t] = cnt;
        tp.ids[t] = b.ids[ids_cur][i];
        static_cast<V4<T>*>(tp.pos)[t] = p;
    }
    uint32_t most = cnt;   // one atomic per wave
    for (int d = 32; d >= 1; d >>= 1) most = max(most, uint32_t(__shfl_xor(int(most), d, 64)));
    if (lane_id() == 0 && most > 0) atomicMax(tp.worst, most);
}

// k_adj_w on a complete tape: F_i and its parameter derivatives from the
// listed contacts, in their order.
template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_tape_w(Buffers<T> b, TapeStep tp, const double* __restrict__ lam,
                                                             double* __restrict__ w) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, n = b.n;
    double gk = 0.0, gg = 0.0;
    if (t < n) {
        const uint32_t i = tp.ids[t], cnt = tp.cnt[t];
        double wi[3] = {0.0, 0.0, 0.0};
        if (i >= n || cnt > kTapeWidth) {
            raise_error(b.g, kErrInternal);
        } else {
            const SimGrid& G = b.sims[0];
            const V4<T>* __restrict__ tpos = static_cast<const V4<T>*>(tp.pos);
            const V4<T> p = tpos[t];
            const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
            const double ri = 0.5 * fabs(double(p.w));
            ForceSum acc;
            for (uint32_t r = 0; r < cnt; ++r) {
                const uint32_t c = tp.list[size_t(r) * n + t];
                add_term<true>(acc, pair_term<T>(xi, yi, zi, ri, tpos[min(c, n - 1u)], G.k, G.gamma));
            }
            adjoint_w(G, acc, lam, i, wi, gk, gg);
        }
        for (int a = 0; a < 3; ++a) w[3 * size_t(t) + a] = wi[a];
    }
    block_partials(b.partials, b.partial_cap, gk, gg);
}

// k_adj_gather on a complete tape: lambda_m + sum_j A_mj (w_m - w_j) over the
// listed contacts, in their order.
template <class T>
__global__ __launch_bounds__(kAdjThreads) void k_adj_tape_gather(Buffers<T> b, TapeStep tp,
                                                                  const double* __restrict__ lam,
                                                                  const double* __restrict__ w,
                                                                  double* __restrict__ lam_out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, n = b.n;
    if (t >= n) return;
    const uint32_t m = tp.ids[t], cnt = tp.cnt[t];
    if (m >= n || cnt > kTapeWidth) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const SimGrid& G = b.sims[0];
    const V4<T>* __restrict__ tpos = static_cast<const V4<T>*>(tp.pos);
    const V4<T> p = tpos[t];
    const double xm = double(p.x), ym = double(p.y), zm = double(p.z);
    const double rm = 0.5 * fabs(double(p.w));
    double acc[3], wm[3];
    for (int a = 0; a < 3; ++a) {
        acc[a] = lam[3 * size_t(m) + a];
        wm[a] = w[3 * size_t(t) + a];
    }
    for (uint32_t r = 0; r < cnt; ++r) {
        const uint32_t c = tp.list[size_t(r) * n + t];
        double o[3];
        gather_term<T>(b, G, xm, ym, zm, rm, wm, w, tpos[min(c, n - 1u)], n + c, o);
        for (int a = 0; a < 3; ++a) acc[a] += o[a];
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

template <class T>
void launch_adj_w(const Buffers<T>& b, int ids_cur, const double* lam, double* w, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_w<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), walk_lds_bytes<kAdjChunk>(kAdjThreads), s, b, ids_cur,
                       lam, w);
}

template <class T>
void launch_adj_gather(const Buffers<T>& b, int ids_cur, const double* lam, const double* w, double* lam_out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adj_gather<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), walk_lds_bytes<kAdjChunk>(kAdjThreads), s, b,
                       ids_cur, lam, w, lam_out);
}

template <class T>
void launch_adj_tape(const Buffers<T>& b, int ids_cur, const TapeStep& tp, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_tape<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), walk_lds_bytes<kAdjChunk>(kAdjThreads), s, b,
                       ids_cur, tp);
}

template <class T>
void launch_adj_tape_w(const Buffers<T>& b, const TapeStep& tp, const double* lam, double* w, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_tape_w<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), 0, s, b, tp, lam, w);
}

template <class T>
void launch_adj_tape_gather(const Buffers<T>& b, const TapeStep& tp, const double* lam, const double* w,
                            double* lam_out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_tape_gather<T>, dim3(adj_blocks(b.n)), dim3(kAdjThreads), 0, s, b, tp, lam, w, lam_out);
}

template <class T>
void launch_adj_finish(const Buffers<T>& b, int nblocks, double* dparams, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_finish, dim3(1), dim3(kAdjThreads), 0, s, b.partials, nblocks, dparams);
}

#define ABM_INSTANTIATE(T)                                                                              \
    template void launch_adj_w<T>(const Buffers<T>&, int, const double*, double*, hipStream_t);       \
    template void launch_adj_gather<T>(const Buffers<T>&, int, const double*, const double*, double*, \
                                       hipStream_t);                                                  \
    template void launch_adj_finish<T>(const Buffers<T>&, int, double*, hipStream_t);                 \
    template void launch_adj_tape<T>(const Buffers<T>&, int, const TapeStep&, hipStream_t);            \
    template void launch_adj_tape_w<T>(const Buffers<T>&, const TapeStep&, const double*, double*,     \
                                       hipStream_t);                                                  \
    template void launch_adj_tape_gather<T>(const Buffers<T>&, const TapeStep&, const double*,         \
                                            const double*, double*, hipStream_t);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
