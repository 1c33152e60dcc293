// force_loop.h -- the 27-box neighbour walk and the pair force, shared by the
// step kernel and the reverse-mode kernels.
//
// The walk reads the slot-ordered copy `spos` that the grid build writes:
// slot u holds {x, y, z, d} of the u-th agent in canonical (box rank, id)
// order, with the sign of d set when that agent moved in the last step.  A
// box's agents are a contiguous slot range, so a candidate costs one load.
#pragma once

#include "abm_device.h"

namespace abm {

template <class T>
__device__ __forceinline__ const V4<T>* spos_ptr(const Buffers<T>& b) {
    return reinterpret_cast<const V4<T>*>(b.spos);
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

// Table entries of the 27 boxes around box q (Section 3.1: the query box and
// its 26 neighbours), in lexicographic (dz, dy, dx) order.  All 27 loads are
// issued before any is used.  Boxes outside the space, and boxes whose entry
// carries another step's stamp (empty this step), read as 0.
template <class T>
__device__ __forceinline__ void load_boxes(const Buffers<T>& b, const SimGrid& G, const uint32_t q[3],
                                           uint32_t stamp, unsigned long long e[27]) {
    const uint32_t dx = G.dims[0], dy = G.dims[1], dz = G.dims[2];
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const int ox = k % 3 - 1, oy = (k / 3) % 3 - 1, oz = k / 9 - 1;
        const int64_t x = int64_t(q[0]) + ox, y = int64_t(q[1]) + oy, z = int64_t(q[2]) + oz;
        const bool in = x >= 0 && x < int64_t(dx) && y >= 0 && y < int64_t(dy) && z >= 0 && z < int64_t(dz);
        const uint32_t idx = G.box_base + (uint32_t(z) * dy + uint32_t(y)) * dx + uint32_t(x);
        e[k] = in ? b.cellinfo[idx] : 0ull;
    }
    const uint32_t st15 = stamp & 0x7FFFu;
#pragma unroll
    for (int k = 0; k < 27; ++k)
        if (cell_stamp_of(e[k]) != st15) e[k] = 0ull;
}

// Visit the slots of the boxes in e (in order; agents of a box in canonical
// order).  With only_moved, boxes without a moved agent are skipped.  fn(slot)
// returns false to stop; visit_slots then returns false.
template <class Fn>
__device__ __forceinline__ bool visit_slots(const unsigned long long e[27], bool only_moved, Fn&& fn) {
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const unsigned long long v = e[k];
        if (only_moved && !cell_moved_of(v)) continue;
        const uint32_t s0 = cell_start_of(v), s1 = s0 + cell_count_of(v);
        for (uint32_t u = s0; u < s1; ++u)
            if (!fn(u)) return false;
    }
    return true;
}

struct ForceSum {
    double fx = 0.0, fy = 0.0, fz = 0.0;   // F_i
    double kx = 0.0, ky = 0.0, kz = 0.0;   // dF_i/dk    = sum_j delta_ij u_ij
    double gx = 0.0, gy = 0.0, gz = 0.0;   // dF_i/dgamma = -sum_j sqrt(rho_ij delta_ij) u_ij
    uint32_t nnz = 0;
};

// F_i over the neighbours j (|e|^2 < R^2) in contact (0 < |e| < r_i + r_j):
// f = k delta - gamma sqrt(rho delta) along e / |e| (the force-law reading of
// Section 5).  Evaluated in double, without fused multiply-adds (the library
// is built with contraction off), in the visiting order of visit_slots.
// `self` is the agent's own slot.
template <class T, bool PARAM_GRADS>
__device__ __forceinline__ void force_of(const Buffers<T>& b, const SimGrid& G, uint32_t self, const V4<T>& p,
                                         const unsigned long long e[27], ForceSum& acc) {
    const V4<T>* __restrict__ sp = spos_ptr(b);
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double ri = 0.5 * fabs(double(p.w));
    const double r2 = G.r2, k = G.k, gamma = G.gamma;
    visit_slots(e, false, [&](uint32_t u) {
        if (u == self || u >= b.n) return true;
        const V4<T> pj = sp[u];
        const double ex = xi - double(pj.x), ey = yi - double(pj.y), ez = zi - double(pj.z);
        const double s2 = (ex * ex + ey * ey) + ez * ez;
        if (!(s2 < r2)) return true;
        const double rj = 0.5 * fabs(double(pj.w));
        const double S = ri + rj;
        if (!(s2 > 0.0) || !(s2 < S * S)) return true;
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
        return true;
    });
}

// Static test of Section 5 for an agent that itself did not move and had at
// most one non-zero pair term: true if no agent within R of it moved.
template <class T>
__device__ __forceinline__ bool no_moved_neighbour(const Buffers<T>& b, const SimGrid& G, uint32_t self,
                                                   const V4<T>& p, const unsigned long long e[27]) {
    const V4<T>* __restrict__ sp = spos_ptr(b);
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double r2 = G.r2;
    return visit_slots(e, true, [&](uint32_t u) {
        if (u == self || u >= b.n) return true;
        const V4<T> pj = sp[u];
        if (!(pj.w < T(0))) return true;   // the sign of d carries the moved flag
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
