// force_loop.h -- the 27-box neighbour walk and the pair force, shared by the
// step kernel and the reverse-mode kernels.
#pragma once

#include "abm_device.h"

namespace abm {

// Visit the agents of the 27 boxes around box q (boxes outside the space are
// skipped; Section 3.1), boxes in lexicographic (dz, dy, dx) order and the
// agents of a box in canonical (id) order.  Boxes whose table entry carries
// another step's stamp are empty.  With only_moved, boxes without a moved
// agent are skipped too.  fn(storage index) returns false to stop the walk;
// visit_boxes then returns false.
template <class T, class Fn>
__device__ __forceinline__ bool visit_boxes(const Buffers<T>& b, const SimGrid& G, const uint32_t q[3],
                                            uint32_t stamp, bool only_moved, Fn&& fn) {
    const uint32_t dx = G.dims[0], dy = G.dims[1], dz = G.dims[2];
    const uint32_t st15 = stamp & 0x7FFFu;
    for (int oz = -1; oz <= 1; ++oz) {
        const int64_t z = int64_t(q[2]) + oz;
        if (z < 0 || z >= int64_t(dz)) continue;
        for (int oy = -1; oy <= 1; ++oy) {
            const int64_t y = int64_t(q[1]) + oy;
            if (y < 0 || y >= int64_t(dy)) continue;
            const uint32_t row = G.box_base + (uint32_t(z) * dy + uint32_t(y)) * dx;
            for (int ox = -1; ox <= 1; ++ox) {
                const int64_t x = int64_t(q[0]) + ox;
                if (x < 0 || x >= int64_t(dx)) continue;
                const unsigned long long e = b.cellinfo[row + uint32_t(x)];
                if (cell_stamp_of(e) != st15) continue;
                if (only_moved && !cell_moved_of(e)) continue;
                const uint32_t s0 = cell_start_of(e), s1 = s0 + cell_count_of(e);
                for (uint32_t u = s0; u < s1; ++u) {
                    const uint32_t j = b.perm[u];
                    if (j < b.n && !fn(j)) return false;
                }
            }
        }
    }
    return true;
}

// Box coordinates of a stored position relative to the simulation's grid.
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

struct ForceSum {
    double fx = 0.0, fy = 0.0, fz = 0.0;   // F_i
    double kx = 0.0, ky = 0.0, kz = 0.0;   // dF_i/dk    = sum_j delta_ij u_ij
    double gx = 0.0, gy = 0.0, gz = 0.0;   // dF_i/dgamma = -sum_j sqrt(rho_ij delta_ij) u_ij
    uint32_t nnz = 0;
};

// F_i over the neighbours j (|e|^2 < R^2) in contact (0 < |e| < r_i + r_j):
// f = k delta - gamma sqrt(rho delta) along e / |e| (the force-law reading of
// Section 5).  Evaluated in double, without fused multiply-adds (the library
// is built with contraction off), in the visiting order of visit_boxes.
template <class T, bool PARAM_GRADS>
__device__ __forceinline__ void force_of(const Buffers<T>& b, const SimGrid& G, const V4<T>* __restrict__ pos,
                                         uint32_t i, const V4<T>& p, const uint32_t q[3], uint32_t stamp,
                                         ForceSum& acc) {
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double ri = 0.5 * double(p.w);
    const double r2 = G.r2, k = G.k, gamma = G.gamma;
    visit_boxes(b, G, q, stamp, false, [&](uint32_t j) {
        if (j == i) return true;
        const V4<T> pj = pos[j];
        const double ex = xi - double(pj.x), ey = yi - double(pj.y), ez = zi - double(pj.z);
        const double s2 = (ex * ex + ey * ey) + ez * ez;
        if (!(s2 < r2)) return true;
        const double rj = 0.5 * double(pj.w);
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
