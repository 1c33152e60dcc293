// force_loop.h -- the neighbour walk and the pair force, shared by the step
// kernel and the reverse-mode kernels.
//
// Agents sit in slots of the canonical (box rank, id) order; the grid build
// writes the slot-ordered copy `spos` ({x, y, z, d}, sign of d = moved in the
// last step).  The walk covers the 3x3x3 boxes of Section 3.1 through
// super-boxes: the aligned 2x2x2 block S = q >> 1 of boxes is 8 consecutive
// Morton codes, so its agents are one contiguous slot range, kept in a
// row-major super-box table (the `cellinfo` array) stamped with the step.
// Along each axis the boxes q-1..q+1 lie in two super-boxes, so 8 ranges
// cover the 27 boxes.  The ranges are disjoint; visited in ascending start
// they yield every neighbour in ascending slot order, the canonical order of
// the sums.  Agents of the 8 super-boxes outside the 27 boxes are rejected by
// the distance test like any other non-neighbour.
#pragma once

#include "abm_device.h"

namespace abm {

template <class T>
__device__ __forceinline__ const V4<T>* spos_ptr(const Buffers<T>& b) {
    return reinterpret_cast<const V4<T>*>(b.spos);
}

// Super-box table entry: start slot (high 32 bits), 15-bit stamp, 17-bit count.
__device__ __forceinline__ unsigned long long pack_super(uint32_t start, uint32_t cnt, uint32_t stamp) {
    return ((unsigned long long)start << 32) | ((unsigned long long)(stamp & 0x7FFFu) << 17) |
           (unsigned long long)(cnt & 0x1FFFFu);
}
__device__ __forceinline__ uint32_t super_start(unsigned long long e) { return uint32_t(e >> 32); }
__device__ __forceinline__ uint32_t super_count(unsigned long long e) { return uint32_t(e) & 0x1FFFFu; }
__device__ __forceinline__ uint32_t super_stamp(unsigned long long e) { return (uint32_t(e) >> 17) & 0x7FFFu; }
constexpr uint32_t kMaxSuperCount = 0x1FFFFu;

__device__ __forceinline__ uint32_t super_dim(uint32_t d) { return (d + 1u) >> 1; }

// Row-major index of super-box (sx, sy, sz) in the simulation's table.
__device__ __forceinline__ uint32_t super_index(const SimGrid& G, uint32_t sx, uint32_t sy, uint32_t sz) {
    return G.box_base + (sz * super_dim(G.dims[1]) + sy) * super_dim(G.dims[0]) + sx;
}

// Ranks of the boxes of q's super-box: [r0, r0 + nin), given q's rank r.
// With w_a in {1, 2} the super-box's in-space width along axis a and b_a the
// low bit of q_a, q's position inside it in Morton order is
// b_x + b_y w_x + b_z w_x w_y.
__device__ __forceinline__ void super_rank_range(const SimGrid& G, const uint32_t q[3], uint32_t r, uint32_t* r0,
                                                 uint32_t* nin) {
    uint32_t w[3];
    for (int a = 0; a < 3; ++a) w[a] = (G.dims[a] - (q[a] & ~1u)) > 1u ? 2u : 1u;
    const uint32_t pre = (q[0] & 1u) + (q[1] & 1u) * w[0] + (q[2] & 1u) * w[0] * w[1];
    *r0 = r - pre;
    *nin = w[0] * w[1] * w[2];
}

// Box coordinates of a position relative to the simulation's grid.
template <class T>
__device__ __forceinline__ bool box_of(const SimGrid& G, const V4<T>& p, uint32_t q[3]) {
    int32_t c[3];
    if (!(box_coord(double(p.x), G.inv_h, &c[0]) && box_coord(double(p.y), G.inv_h, &c[1]) &&
          box_coord(double(p.z), G.inv_h, &c[2])))
        return false;
    bool in = true;
    for (int a = 0; a < 3; ++a) {
        const int64_t v = int64_t(c[a]) - int64_t(G.cmin[a]);
        in = in && v >= 0 && v < int64_t(G.dims[a]);
        q[a] = uint32_t(v);
    }
    return in;
}

__device__ __forceinline__ void cswap(unsigned long long& a, unsigned long long& b) {
    const unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// The 8 super-box ranges around box q, sorted by start slot; empty or
// out-of-space super-boxes read as 0 (no slots).
template <class T>
__device__ __forceinline__ void load_ranges(const Buffers<T>& b, const SimGrid& G, const uint32_t q[3],
                                            uint32_t stamp, unsigned long long e[8]) {
    const uint32_t sd[3] = {super_dim(G.dims[0]), super_dim(G.dims[1]), super_dim(G.dims[2])};
    uint32_t lo[3];
    for (int a = 0; a < 3; ++a) lo[a] = (q[a] >> 1) - 1u + (q[a] & 1u);   // may wrap: then out of range
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t sx = lo[0] + (k & 1), sy = lo[1] + ((k >> 1) & 1), sz = lo[2] + (k >> 2);
        const bool in = sx < sd[0] && sy < sd[1] && sz < sd[2];
        e[k] = in ? b.cellinfo[G.box_base + (sz * sd[1] + sy) * sd[0] + sx] : 0ull;
    }
    const uint32_t st15 = stamp & 0x7FFFu;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (super_stamp(e[k]) != st15) e[k] = 0ull;
    cswap(e[0], e[2]); cswap(e[1], e[3]); cswap(e[4], e[6]); cswap(e[5], e[7]);
    cswap(e[0], e[4]); cswap(e[1], e[5]); cswap(e[2], e[6]); cswap(e[3], e[7]);
    cswap(e[0], e[1]); cswap(e[2], e[3]); cswap(e[4], e[5]); cswap(e[6], e[7]);
    cswap(e[2], e[4]); cswap(e[3], e[5]);
    cswap(e[1], e[4]); cswap(e[3], e[6]);
    cswap(e[1], e[2]); cswap(e[3], e[4]); cswap(e[5], e[6]);
}

// Visit the slots of the sorted ranges in ascending order.  fn(slot) returns
// false to stop; visit_ranges then returns false.
template <class Fn>
__device__ __forceinline__ bool visit_ranges(const unsigned long long e[8], Fn&& fn) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t s0 = super_start(e[k]), s1 = s0 + super_count(e[k]);
        for (uint32_t u = s0; u < s1; ++u)
            if (!fn(u)) return false;
    }
    return true;
}

// Per-thread scratch in LDS for the neighbour walk: the 8 sorted ranges and a
// queue of candidate slots.  Laid out [entry][thread] so that the threads of
// a wave hit distinct banks.
constexpr int kQueueCap = 8;
struct WalkLds {
    unsigned long long* rng;   // [8][blockDim]
    uint32_t* queue;           // [kQueueCap][blockDim]
};
inline size_t walk_lds_bytes(int block) { return size_t(block) * (8 * 8 + kQueueCap * 4); }

__device__ __forceinline__ WalkLds walk_lds(void* base) {
    WalkLds w;
    w.rng = static_cast<unsigned long long*>(base);
    w.queue = reinterpret_cast<uint32_t*>(w.rng + 8 * blockDim.x);
    return w;
}

// The slots of the sorted ranges as one stream in ascending order.  Each lane
// advances through its own ranges (read back from LDS), so a wave iterates
// max(total) times rather than the sum of per-range maxima.  fn(slot) returns
// false to stop; stream_slots then returns false.
template <class Fn>
__device__ __forceinline__ bool stream_slots(const unsigned long long e[8], const WalkLds& L, Fn&& fn) {
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        total += super_count(e[k]);
        L.rng[k * bs + tid] = e[k];
    }
    int k = -1;
    uint32_t u = 0, end = 0;
    for (uint32_t j = 0; j < total; ++j) {
        while (u >= end && k < 7) {   // next non-empty range
            ++k;
            const unsigned long long v = L.rng[k * bs + tid];
            u = super_start(v);
            end = u + super_count(v);
        }
        if (!fn(u)) return false;
        ++u;
    }
    return true;
}

// Conservative single-precision pre-test of |x_i - x_j|^2 < R^2 for float
// state: false only if the exact double test must fail (the float sum of
// squares is within a few ulp of the exact value; the bound is padded by
// 2^-16 relative).  Double state goes straight to the exact test.
template <class T>
__device__ __forceinline__ bool maybe_within(const V4<T>& pi, const V4<T>& pj, float r2pad) {
    if constexpr (sizeof(T) == 4) {
        const float ex = pi.x - pj.x, ey = pi.y - pj.y, ez = pi.z - pj.z;
        return __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)) < r2pad;
    } else {
        return true;
    }
}

__device__ __forceinline__ float padded_r2(double r2) { return float(r2 * (1.0 + 1.0 / 65536.0)) * 1.0001f; }

struct ForceSum {
    double fx = 0.0, fy = 0.0, fz = 0.0;   // F_i
    double kx = 0.0, ky = 0.0, kz = 0.0;   // dF_i/dk    = sum_j delta_ij u_ij
    double gx = 0.0, gy = 0.0, gz = 0.0;   // dF_i/dgamma = -sum_j sqrt(rho_ij delta_ij) u_ij
    uint32_t nnz = 0;
};

// F_i over the neighbours j (|e|^2 < R^2) in contact (0 < |e| < r_i + r_j):
// f = k delta - gamma sqrt(rho delta) along e / |e| (the force-law reading of
// Section 5).  Evaluated in double, without fused multiply-adds (the library
// is built with contraction off), in ascending slot order.  `self` is the
// agent's own slot.
//
// Pass 1 streams the candidates through the cheap pre-test and queues the
// survivors; a full queue (and the end) is drained by pass 2, which keeps the
// candidates in contact (exact test, in place) and then adds their terms.
// Queue order is stream order, so the terms are summed in ascending slot
// order.
template <class T, bool PARAM_GRADS>
__device__ __forceinline__ void force_of(const Buffers<T>& b, const SimGrid& G, uint32_t self, const V4<T>& p,
                                         const unsigned long long e[8], const WalkLds& L, ForceSum& acc) {
    const V4<T>* __restrict__ sp = spos_ptr(b);
    const uint32_t tid = threadIdx.x, bs = blockDim.x, last = b.n - 1;
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double ri = 0.5 * fabs(double(p.w));
    const double r2 = G.r2, k = G.k, gamma = G.gamma;
    const float r2pad = padded_r2(r2);
    uint32_t n = 0;
    auto drain = [&]() {
        // exact neighbour + contact test, keeping the survivors in place; the
        // positions of a group of four are requested before any is tested
        uint32_t m = 0;
        for (uint32_t x0 = 0; x0 < n; x0 += 4) {
            V4<T> pj[4];
            uint32_t uq[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uq[c] = L.queue[min(x0 + c, n - 1) * bs + tid];
                pj[c] = sp[uq[c]];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double ex = xi - double(pj[c].x), ey = yi - double(pj[c].y), ez = zi - double(pj[c].z);
                const double s2 = (ex * ex + ey * ey) + ez * ez;
                const double S = ri + 0.5 * fabs(double(pj[c].w));
                const bool keep = x0 + c < n && s2 < r2 && s2 > 0.0 && s2 < S * S;
                L.queue[m * bs + tid] = uq[c];
                m += keep ? 1u : 0u;
            }
        }
        for (uint32_t x = 0; x < m; ++x) {   // pair terms, in slot order
            const V4<T> pj = sp[L.queue[x * bs + tid]];
            const double ex = xi - double(pj.x), ey = yi - double(pj.y), ez = zi - double(pj.z);
            const double s2 = (ex * ex + ey * ey) + ez * ez;
            const double rj = 0.5 * fabs(double(pj.w));
            const double S = ri + rj;
            const double dist = sqrt(s2);
            const double delta = S - dist;
            const double rho = (ri * rj) / S;
            const double sr = sqrt(rho * delta);
            const double f = k * delta - gamma * sr;
            const double sc = f / dist;
            acc.fx += sc * ex;
            acc.fy += sc * ey;
            acc.fz += sc * ez;
            acc.nnz += f != 0.0 ? 1u : 0u;
            if (PARAM_GRADS) {
                const double ux = ex / dist, uy = ey / dist, uz = ez / dist;
                acc.kx += delta * ux;
                acc.ky += delta * uy;
                acc.kz += delta * uz;
                acc.gx -= sr * ux;
                acc.gy -= sr * uy;
                acc.gz -= sr * uz;
            }
        }
        n = 0;
    };
    // pass 1: stream the candidates through the pre-test, the next
    // candidate's position requested one iteration ahead
    uint32_t total = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        total += super_count(e[q]);
        L.rng[q * bs + tid] = e[q];
    }
    int kr = -1;
    uint32_t u = 0, end = 0;
    auto advance = [&]() {
        while (u >= end && kr < 7) {
            ++kr;
            const unsigned long long v = L.rng[kr * bs + tid];
            u = super_start(v);
            end = u + super_count(v);
        }
    };
    advance();
    V4<T> pn = sp[min(u, last)];
    for (uint32_t j = 0; j < total; ++j) {
        const uint32_t uc = u;
        const V4<T> pc = pn;
        ++u;
        advance();
        pn = sp[min(u, last)];
        const bool pass = uc != self && maybe_within<T>(p, pc, r2pad);
        L.queue[n * bs + tid] = uc;   // n < kQueueCap here
        n += pass ? 1u : 0u;
        if (n == uint32_t(kQueueCap)) drain();
    }
    drain();
}

// Static test of Section 5 for an agent that itself did not move and had at
// most one non-zero pair term: true if no agent within R of it moved.
template <class T>
__device__ __forceinline__ bool no_moved_neighbour(const Buffers<T>& b, const SimGrid& G, uint32_t self,
                                                   const V4<T>& p, const unsigned long long e[8],
                                                   const WalkLds& L) {
    const V4<T>* __restrict__ sp = spos_ptr(b);
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double r2 = G.r2;
    const float r2pad = padded_r2(r2);
    return stream_slots(e, L, [&](uint32_t u) {
        if (u == self || u >= b.n) return true;
        const V4<T> pj = sp[u];
        if (!(pj.w < T(0))) return true;   // the sign of d carries the moved flag
        if (!maybe_within<T>(p, pj, r2pad)) return true;
        const double ex = xi - double(pj.x), ey = yi - double(pj.y), ez = zi - double(pj.z);
        return !(((ex * ex + ey * ey) + ez * ez) < r2);
    });
}

// Displacement rule: Delta = mu F if |F| > f_adh, clamped to delta_max.
struct Move {
    double ux = 0.0, uy = 0.0, uz = 0.0;
    bool moves = false;
    bool clamped = false;
    double fnorm = 0.0;
};

__device__ __forceinline__ Move displacement(const SimGrid& G, double fx, double fy, double fz) {
    Move m;
    m.fnorm = sqrt((fx * fx + fy * fy) + fz * fz);
    if (m.fnorm > G.f_adh) {
        m.moves = true;
        m.ux = G.mu * fx;
        m.uy = G.mu * fy;
        m.uz = G.mu * fz;
        const double un = sqrt((m.ux * m.ux + m.uy * m.uy) + m.uz * m.uz);
        if (un > G.delta_max) {
            const double s = G.delta_max / un;
            m.ux *= s;
            m.uy *= s;
            m.uz *= s;
            m.clamped = true;
        }
    }
    return m;
}

}  // namespace abm
