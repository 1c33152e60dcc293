// abm_oracle.cpp -- CPU oracle for one mechanical step of N spherical agents.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference that the GPU path is checked against.  Only the tests, the smoke
// check and the benchmark's CPU-baseline leg may load it; the product library
// never links, loads or calls it, and it shares no source with the GPU path.
//
// What it computes, and where the paper defines it:
//  * Uniform grid with a 3x3x3 box search (Section 3.1): an agent's box is a
//    constant-time function of its position, the neighbour candidates are the
//    agents of the 27 boxes around it, each box holds an array-based list
//    (start index + count).
//  * Gap-free Morton ranks of the boxes (Section 4.2, steps D and E): a
//    depth-first walk of the implicit 2^D-ary tree over the power-of-two cube
//    produces a sorted table of (box counter, offset) entries; Morton code =
//    rank + offset of the entry that covers the rank.
//  * A variant order (Section 4.2 compares Morton order with the Hilbert
//    curve): the 2x2x2 blocks of boxes follow a Hilbert curve (Skilling's
//    transform), the boxes inside a block Morton order; ranks by brute force.
//  * Static agents (Section 5): the force of an agent is skipped when it and
//    none of its neighbours moved in the last iteration and at most one
//    neighbour force was non-zero.
//  * Displacement from the summed force with a force threshold (Section 5).
//  * Sums over neighbours run in canonical (box rank, id) order.
//  * Parallel-for over agents with a barrier before positions are committed
//    (Algorithm 1), read as a Jacobi update.
// The pairwise force law is not given in the paper (Section 5 defers to the
// Cortex3D method); the reading used here is
//     f(delta, rho) = k*delta - gamma*sqrt(rho*delta)
// acting along the centre line, with delta the overlap and rho the reduced
// radius r_i r_j / (r_i + r_j).  Displacement is overdamped: mu * F, applied
// only when |F| exceeds the threshold, clamped to delta_max.
//
// Arithmetic: every geometric decision (box coordinate, radius test, contact
// test) and the force are evaluated in IEEE double from the stored positions
// promoted exactly to double; no fused multiply-add (built with
// -ffp-contract=off).  Only the final position is rounded to the storage
// type T.  Integer results (box keys, order, neighbour sets) therefore depend
// on T only through the stored positions.
//
// Parity status: gap table, keys, order, neighbour sets, pair force, static
// rule and displacement are pinned by the CPU tests (paper example, brute
// force, closed forms, invariants).  Agreement with BioDynaMo's own force
// implementation is unpinned: the paper does not print its force law.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <tuple>
#include <utility>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

struct orc_params {
    double k;                   // repulsion coefficient
    double gamma;               // adhesion coefficient
    double mu;                  // mobility: displacement per unit force
    double f_adh;               // force threshold that must be exceeded to move
    double delta_max;           // largest displacement per step
    double interaction_radius;  // 0: the largest diameter
    double cell_factor;         // box edge = cell_factor * interaction radius (>= 1)
    int32_t detect_static;      // skip the force of static agents
    int32_t nthreads;           // OpenMP threads, 0 = runtime default
    int32_t order;              // 0: Morton order of the boxes; 1: Hilbert order of the 2x2x2 blocks
};

}  // extern "C"

namespace {

constexpr int64_t kMaxDim = int64_t(1) << 21;

int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

int levels_for(const int64_t* dims, int D) {
    int64_t m = 1;
    for (int a = 0; a < D; ++a) m = std::max(m, dims[a]);
    int L = 0;
    while ((int64_t(1) << L) < m) ++L;
    return L;
}

// Morton code: bit D*b + a holds bit b of coordinate a (x in the lowest bit).
uint64_t morton(const int64_t* q, int D, int L) {
    uint64_t m = 0;
    for (int b = 0; b < L; ++b)
        for (int a = 0; a < D; ++a)
            m |= uint64_t((q[a] >> b) & 1) << (D * b + a);
    return m;
}

// ---- Section 4.2, step D: gaps between the boxes of the simulation space
// in Morton order, from a depth-first walk of the implicit tree.
struct GapWalk {
    int D;
    int64_t dims[3];
    int64_t box_counter = 0;
    int64_t offset = 0;
    bool found_gap = true;
    std::vector<int64_t> e_counter, e_offset;

    void visit(const int64_t* origin, int64_t size) {
        int64_t inside = 1, total = 1;
        for (int a = 0; a < D; ++a) {
            inside *= clamp64(dims[a] - origin[a], 0, size);
            total *= size;
        }
        if (inside == 0) {             // empty node or empty leaf
            offset += total;
            found_gap = true;
            return;
        }
        if (inside == total) {         // complete node or leaf inside the space
            if (found_gap) {
                e_counter.push_back(box_counter);
                e_offset.push_back(offset);
                found_gap = false;
            }
            box_counter += total;
            return;
        }
        const int64_t half = size / 2;  // partial node: descend in Morton order
        for (int c = 0; c < (1 << D); ++c) {
            int64_t child[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) child[a] = origin[a] + (((c >> a) & 1) ? half : 0);
            visit(child, half);
        }
    }
};

struct GapTable {
    std::vector<int64_t> counter, offset;  // sorted by counter
    int D = 3, L = 0;
};

GapTable build_gap_table(const int64_t* dims, int D) {
    GapWalk w;
    w.D = D;
    for (int a = 0; a < 3; ++a) w.dims[a] = a < D ? dims[a] : 1;
    const int L = levels_for(dims, D);
    const int64_t origin[3] = {0, 0, 0};
    w.visit(origin, int64_t(1) << L);
    GapTable t;
    t.counter = std::move(w.e_counter);
    t.offset = std::move(w.e_offset);
    t.D = D;
    t.L = L;
    return t;
}

// Step E, inverted: Morton code of a box inside the space -> its rank.  The
// covering entry is the last one whose first code (counter + offset) <= m.
int64_t rank_of_code(const GapTable& t, uint64_t m) {
    int64_t lo = 0, hi = int64_t(t.counter.size()) - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (uint64_t(t.counter[mid] + t.offset[mid]) <= m) lo = mid; else hi = mid - 1;
    }
    return int64_t(m) - t.offset[lo];
}

// Step E: rank -> Morton code, using the last entry whose counter <= rank.
uint64_t code_of_rank(const GapTable& t, int64_t r) {
    int64_t lo = 0, hi = int64_t(t.counter.size()) - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (t.counter[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return uint64_t(r + t.offset[lo]);
}

// ---- Section 4.2 names the Hilbert curve as the other space-filling curve
// it compared with Morton order.  The variant here orders the aligned 2x2x2
// blocks of boxes ("super-boxes") along a Hilbert curve and keeps Morton
// order among the 8 boxes of a block.
//
// Hilbert index of a lattice point with coordinates below 2^b, by Skilling's
// transform (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc.
// 707, 2004): from the top bit level down, the lower bits of the first
// coordinate are inverted or exchanged with those of each coordinate in turn
// (undoing the rotations of the recursive construction), then the
// coordinates are Gray-encoded into the "transposed" index.  The index reads
// its bits level by level from the top, the first coordinate's bit first.
uint64_t hilbert_index(const int64_t* q, int b) {
    if (b <= 0) return 0;
    uint64_t X[3] = {uint64_t(q[0]), uint64_t(q[1]), uint64_t(q[2])};
    const uint64_t M = uint64_t(1) << (b - 1);
    for (uint64_t Q = M; Q > 1; Q >>= 1) {
        const uint64_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint64_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint64_t t = 0;
    for (uint64_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int lev = b - 1; lev >= 0; --lev)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> lev) & 1);
    return h;
}

// Rank of every box (indexed x fastest) in the Hilbert variant, by brute
// force: the super-boxes that meet the space sorted by Hilbert index over the
// smallest power-of-two cube that holds them, then the boxes inside the
// space of each super-box in Morton order (x lowest), counted consecutively.
std::vector<uint32_t> hilbert_box_ranks(const int64_t* dims) {
    int64_t sd[3];
    for (int a = 0; a < 3; ++a) sd[a] = (dims[a] + 1) / 2;
    const int L = levels_for(sd, 3);
    std::vector<std::pair<uint64_t, int64_t>> order;
    order.reserve(size_t(sd[0] * sd[1] * sd[2]));
    for (int64_t z = 0; z < sd[2]; ++z)
        for (int64_t y = 0; y < sd[1]; ++y)
            for (int64_t x = 0; x < sd[0]; ++x) {
                const int64_t S[3] = {x, y, z};
                order.push_back({hilbert_index(S, L), (z * sd[1] + y) * sd[0] + x});
            }
    std::sort(order.begin(), order.end());
    std::vector<uint32_t> rank(size_t(dims[0] * dims[1] * dims[2]), 0xFFFFFFFFu);
    uint32_t r = 0;
    for (const auto& e : order) {
        const int64_t S[3] = {e.second % sd[0], (e.second / sd[0]) % sd[1], e.second / (sd[0] * sd[1])};
        for (int c = 0; c < 8; ++c) {
            const int64_t q[3] = {2 * S[0] + (c & 1), 2 * S[1] + ((c >> 1) & 1), 2 * S[2] + ((c >> 2) & 1)};
            if (q[0] < dims[0] && q[1] < dims[1] && q[2] < dims[2]) rank[size_t((q[2] * dims[1] + q[1]) * dims[0] + q[0])] = r++;
        }
    }
    return rank;
}

// ---- Section 3.1: the uniform grid.
template <class T>
struct Grid {
    int64_t n = 0;
    double inv_h = 0;
    int64_t cmin[3] = {0, 0, 0}, dims[3] = {1, 1, 1};
    int64_t nboxes = 0;
    GapTable table;
    int order = 0;                      // 0: Morton; 1: Hilbert order of the super-boxes
    std::vector<uint32_t> hrank;        // order 1: rank of every box (x fastest)
    std::vector<int64_t> cell;          // per agent: 3 box coordinates relative to cmin
    std::vector<uint32_t> key;          // per agent: gap-free rank of its box in the grid's order
    std::vector<uint32_t> perm;         // slot -> agent id, ordered by (key, id)
    std::vector<uint32_t> cell_start;   // nboxes + 1 (exclusive prefix sum of counts)

    int64_t box_rank(const int64_t* q) const {
        if (order == 1) return hrank[size_t((q[2] * dims[1] + q[1]) * dims[0] + q[0])];
        return rank_of_code(table, morton(q, 3, table.L));
    }
};

template <class T>
int build_grid(Grid<T>& g, int64_t n, const T* pos, double inv_h, int order = 0) {
    g.n = n;
    g.inv_h = inv_h;
    std::vector<int64_t> c(3 * n);
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double v = double(pos[3 * i + a]) * inv_h;
            if (!std::isfinite(v)) return -2;
            const int64_t ci = int64_t(std::floor(v));
            c[3 * i + a] = ci;
            lo[a] = std::min(lo[a], ci);
            hi[a] = std::max(hi[a], ci);
        }
    g.nboxes = 1;
    for (int a = 0; a < 3; ++a) {
        g.cmin[a] = lo[a];
        g.dims[a] = hi[a] - lo[a] + 1;
        if (g.dims[a] > kMaxDim) return -3;
        g.nboxes *= g.dims[a];
    }
    if (g.nboxes > (int64_t(1) << 32) - 1) return -3;
    g.order = order;
    if (order == 1)
        g.hrank = hilbert_box_ranks(g.dims);
    else
        g.table = build_gap_table(g.dims, 3);
    g.cell.resize(3 * n);
    g.key.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) g.cell[3 * i + a] = c[3 * i + a] - g.cmin[a];
        g.key[i] = uint32_t(g.box_rank(&g.cell[3 * i]));
    }
    // Array-based lists: agents ordered by (box, id); start index per box.
    std::vector<std::pair<uint32_t, uint32_t>> kv(n);
    for (int64_t i = 0; i < n; ++i) kv[i] = {g.key[i], uint32_t(i)};
    std::sort(kv.begin(), kv.end());
    g.perm.resize(n);
    for (int64_t s = 0; s < n; ++s) g.perm[s] = kv[s].second;
    std::vector<uint32_t> count(g.nboxes, 0);
    for (int64_t i = 0; i < n; ++i) count[g.key[i]]++;
    g.cell_start.assign(g.nboxes + 1, 0);
    for (int64_t b = 0; b < g.nboxes; ++b) g.cell_start[b + 1] = g.cell_start[b] + count[b];
    return 0;
}

struct Vec3 { double x, y, z; };

template <class T>
Vec3 load(const T* pos, int64_t i) { return {double(pos[3 * i]), double(pos[3 * i + 1]), double(pos[3 * i + 2])}; }

// Visit the candidates of agent i: the agents of the 27 boxes around its box
// (boxes outside the space are skipped), boxes in lexicographic (dz, dy, dx)
// order, agents of a box in ascending id.  fn(j) is called for j != i.
// The candidates are visited in canonical order: ascending (box rank, id),
// i.e. by their slot in the array-based lists.  Floating-point sums over
// neighbours therefore have one defined order (the paper leaves it open).
template <class T, class Fn>
void for_candidates(const Grid<T>& g, int64_t i, Fn&& fn) {
    const int64_t* q = &g.cell[3 * i];
    std::vector<uint32_t> slots;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t qq[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                bool in = true;
                for (int a = 0; a < 3; ++a) in = in && qq[a] >= 0 && qq[a] < g.dims[a];
                if (!in) continue;
                const int64_t b = g.box_rank(qq);
                for (uint32_t s = g.cell_start[b]; s < g.cell_start[b + 1]; ++s) slots.push_back(s);
            }
    std::sort(slots.begin(), slots.end());
    for (uint32_t s : slots) {
        const uint32_t j = g.perm[s];
        if (int64_t(j) != i) fn(int64_t(j));
    }
}

double sq3(double a, double b, double c) { return (a * a + b * b) + c * c; }

// Pair force law (reading of Section 5; see the file header).
struct PairTerm { bool contact; double f; double fx, fy, fz; };

PairTerm pair_term(const Vec3& xi, double di, const Vec3& xj, double dj, double k, double gamma) {
    PairTerm t{false, 0.0, 0.0, 0.0, 0.0};
    const double ex = xi.x - xj.x, ey = xi.y - xj.y, ez = xi.z - xj.z;
    const double s2 = sq3(ex, ey, ez);
    const double ri = 0.5 * di, rj = 0.5 * dj;
    const double S = ri + rj;
    if (!(s2 > 0.0) || !(s2 < S * S)) return t;
    const double dist = std::sqrt(s2);
    const double delta = S - dist;
    const double rho = (ri * rj) / S;
    const double f = k * delta - gamma * std::sqrt(rho * delta);
    const double scale = f / dist;
    t.contact = true;
    t.f = f;
    t.fx = scale * ex;
    t.fy = scale * ey;
    t.fz = scale * ez;
    return t;
}

double radius_of(int64_t n, const double* d_as_double, const orc_params* p) {
    if (p->interaction_radius > 0) return p->interaction_radius;
    double R = 0.0;
    for (int64_t i = 0; i < n; ++i) R = std::max(R, d_as_double[i]);
    return R;
}

template <class T>
std::vector<double> promote(int64_t n, const T* v) {
    std::vector<double> out(n);
    for (int64_t i = 0; i < n; ++i) out[i] = double(v[i]);
    return out;
}

// Displacement from the summed force (Section 5): mu F when |F| exceeds the
// threshold, clamped to delta_max; otherwise none.
Vec3 displacement(double Fx, double Fy, double Fz, const orc_params* p) {
    if (!(std::sqrt(sq3(Fx, Fy, Fz)) > p->f_adh)) return Vec3{0.0, 0.0, 0.0};
    double ux = p->mu * Fx, uy = p->mu * Fy, uz = p->mu * Fz;
    const double un = std::sqrt(sq3(ux, uy, uz));
    if (un > p->delta_max) {
        const double s = p->delta_max / un;
        ux *= s;
        uy *= s;
        uz *= s;
    }
    return Vec3{ux, uy, uz};
}

template <class T>
int step_impl(int64_t n, T* pos, const T* diam, uint8_t* moved, int32_t* nnz, double* force,
              int64_t t, const orc_params* p, uint8_t* is_static, double* disp) {
    if (n <= 0) return -1;
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
    const std::vector<double> d = promote(n, diam);
    const double R = radius_of(n, d.data(), p);
    const double h = R * (p->cell_factor >= 1.0 ? p->cell_factor : 1.0);
    const double inv_h = 1.0 / h;
    const double R2 = R * R;
    Grid<T> g;
    const int rc = build_grid(g, n, pos, inv_h, p->order);
    if (rc != 0) return rc;

    // Section 5: static agents, decided from the last iteration's state.
    std::vector<uint8_t> st(n, 0);
    if (p->detect_static && t > 0) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if (moved[i] || nnz[i] > 1) continue;
            const Vec3 xi = load(pos, i);
            bool neighbour_moved = false;
            for_candidates(g, i, [&](int64_t j) {
                if (!moved[j]) return;
                const Vec3 xj = load(pos, j);
                if (sq3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z) < R2) neighbour_moved = true;
            });
            st[i] = neighbour_moved ? 0 : 1;
        }
    }

    // Forces of the non-static agents (gather over the neighbour set).
    std::vector<Vec3> dx(n, Vec3{0.0, 0.0, 0.0});
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (st[i]) continue;
        const Vec3 xi = load(pos, i);
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        int32_t cnt = 0;
        for_candidates(g, i, [&](int64_t j) {
            const Vec3 xj = load(pos, j);
            if (!(sq3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z) < R2)) return;
            const PairTerm pt = pair_term(xi, d[i], xj, d[j], p->k, p->gamma);
            if (!pt.contact) return;
            Fx += pt.fx;
            Fy += pt.fy;
            Fz += pt.fz;
            if (pt.f != 0.0) ++cnt;
        });
        force[3 * i] = Fx;
        force[3 * i + 1] = Fy;
        force[3 * i + 2] = Fz;
        nnz[i] = cnt;
        dx[i] = displacement(Fx, Fy, Fz, p);
    }

    // Commit after every force is known (the barrier of Algorithm 1).
    for (int64_t i = 0; i < n; ++i) {
        const Vec3 xi = load(pos, i);
        const bool m = dx[i].x != 0.0 || dx[i].y != 0.0 || dx[i].z != 0.0;
        pos[3 * i] = T(xi.x + dx[i].x);
        pos[3 * i + 1] = T(xi.y + dx[i].y);
        pos[3 * i + 2] = T(xi.z + dx[i].z);
        moved[i] = m ? 1 : 0;
        if (is_static) is_static[i] = st[i];
        if (disp) {
            disp[3 * i] = dx[i].x;
            disp[3 * i + 1] = dx[i].y;
            disp[3 * i + 2] = dx[i].z;
        }
    }
    return 0;
}

template <class T>
int64_t grid_impl(int64_t n, const T* pos, double inv_h, int64_t* cmin, int64_t* dims, uint32_t* key,
                  uint32_t* perm, uint32_t* cell_start, int64_t cell_cap, int order) {
    Grid<T> g;
    const int rc = build_grid(g, n, pos, inv_h, order);
    if (rc != 0) return rc;
    for (int a = 0; a < 3; ++a) {
        cmin[a] = g.cmin[a];
        dims[a] = g.dims[a];
    }
    if (key) std::memcpy(key, g.key.data(), n * sizeof(uint32_t));
    if (perm) std::memcpy(perm, g.perm.data(), n * sizeof(uint32_t));
    if (cell_start) {
        if (g.nboxes + 1 > cell_cap) return -4;
        std::memcpy(cell_start, g.cell_start.data(), (g.nboxes + 1) * sizeof(uint32_t));
    }
    return g.nboxes;
}

// Neighbour sets N(i) = { j != i in the 27 boxes : |x_i - x_j|^2 < R^2 },
// as a CSR with ascending ids per agent.
template <class T>
int64_t neighbors_impl(int64_t n, const T* pos, double R, double inv_h, int64_t* start, uint32_t* nbr,
                       int64_t cap) {
    Grid<T> g;
    const int rc = build_grid(g, n, pos, inv_h);
    if (rc != 0) return rc;
    const double R2 = R * R;
    std::vector<std::vector<uint32_t>> lists(n);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const Vec3 xi = load(pos, i);
        for_candidates(g, i, [&](int64_t j) {
            const Vec3 xj = load(pos, j);
            if (sq3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z) < R2) lists[i].push_back(uint32_t(j));
        });
        std::sort(lists[i].begin(), lists[i].end());
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        start[i] = total;
        for (uint32_t j : lists[i]) {
            if (total < cap) nbr[total] = j;
            ++total;
        }
    }
    start[n] = total;
    return total;
}

// One step for a few sampled agents from the plain definition, without the
// grid: the neighbour set of agent i is every j != i with
// |x_i - x_j|^2 < R^2, found by scanning all agents.  The pair terms are
// added one after another in canonical order (box rank, then id), the order
// the step sums in: ranks are gap-free, so two boxes compare by their Morton
// code relative to the smallest box (the Hilbert order: by the Hilbert index
// of their 2x2x2 block over the smallest power-of-two cube holding the
// blocks, then the octant).  No static skipping (a first step).  The scan
// over the agents may run on several threads; the sum does not, so the
// result does not depend on the thread count.
template <class T>
int sample_impl(int64_t n, const T* pos, const T* diam, const orc_params* p, int64_t ns, const int64_t* ids,
                double* F, int32_t* nnz, T* new_pos) {
    if (n <= 0 || ns < 0) return -1;
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
    const std::vector<double> d = promote(n, diam);
    const double R = radius_of(n, d.data(), p);
    const double R2 = R * R;
    const double inv_h = 1.0 / (R * (p->cell_factor >= 1.0 ? p->cell_factor : 1.0));
    for (int64_t s = 0; s < ns; ++s)
        if (ids[s] < 0 || ids[s] >= n) return -1;
    // the box of every agent, counted from the smallest box per axis
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double v = double(pos[3 * i + a]) * inv_h;
            if (!std::isfinite(v)) return -2;
            const int64_t c = int64_t(std::floor(v));
            lo[a] = std::min(lo[a], c);
            hi[a] = std::max(hi[a], c);
        }
    int64_t sd[3];
    for (int a = 0; a < 3; ++a) sd[a] = (hi[a] - lo[a] + 2) / 2;
    const int sL = levels_for(sd, 3);
    // sort key of agent j's box: monotone in its rank in the grid's order
    auto box_key = [&](int64_t j) -> std::pair<uint64_t, uint32_t> {
        int64_t q[3];
        for (int a = 0; a < 3; ++a) q[a] = int64_t(std::floor(double(pos[3 * j + a]) * inv_h)) - lo[a];
        if (p->order == 1) {
            const int64_t S[3] = {q[0] >> 1, q[1] >> 1, q[2] >> 1};
            return {hilbert_index(S, sL), uint32_t((q[0] & 1) | ((q[1] & 1) << 1) | ((q[2] & 1) << 2))};
        }
        return {morton(q, 3, 21), 0u};
    };
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t i = ids[s];
        const Vec3 xi = load(pos, i);
        // the neighbours in contact, found in any order
        std::vector<int64_t> found;
#pragma omp parallel
        {
            std::vector<int64_t> mine;
#pragma omp for schedule(static) nowait
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                const Vec3 xj = load(pos, j);
                if (!(sq3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z) < R2)) continue;
                if (pair_term(xi, d[i], xj, d[j], p->k, p->gamma).contact) mine.push_back(j);
            }
#pragma omp critical
            found.insert(found.end(), mine.begin(), mine.end());
        }
        // ... put in canonical order and summed one after another
        std::vector<std::tuple<uint64_t, uint32_t, int64_t>> ord;
        ord.reserve(found.size());
        for (int64_t j : found) {
            const auto k = box_key(j);
            ord.emplace_back(k.first, k.second, j);
        }
        std::sort(ord.begin(), ord.end());
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        int32_t cnt = 0;
        for (const auto& e : ord) {
            const int64_t j = std::get<2>(e);
            const PairTerm pt = pair_term(xi, d[i], load(pos, j), d[j], p->k, p->gamma);
            Fx += pt.fx;
            Fy += pt.fy;
            Fz += pt.fz;
            if (pt.f != 0.0) ++cnt;
        }
        F[3 * s] = Fx;
        F[3 * s + 1] = Fy;
        F[3 * s + 2] = Fz;
        nnz[s] = cnt;
        const Vec3 u = displacement(Fx, Fy, Fz, p);
        new_pos[3 * s] = T(xi.x + u.x);
        new_pos[3 * s + 1] = T(xi.y + u.y);
        new_pos[3 * s + 2] = T(xi.z + u.z);
    }
    return 0;
}

// ---- Reverse mode of the step map x -> x + Delta(F(x); k, gamma), with the
// neighbour sets, thresholds and clamp states of each forward step held fixed.
// Static skipping is off on this path.
struct Mat3 { double a[3][3]; };

template <class T>
int adjoint_impl(int64_t n, const T* pos0, const T* diam, int32_t nsteps, const orc_params* p,
                 const double* target, T* posT, double* loss, double* dL_dx0, double* dL_dparams) {
    if (n <= 0 || nsteps < 0) return -1;
    if (p->detect_static) return -7;
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
    const std::vector<double> d = promote(n, diam);
    const double R = radius_of(n, d.data(), p);
    const double inv_h = 1.0 / (R * (p->cell_factor >= 1.0 ? p->cell_factor : 1.0));
    // forward, keeping every intermediate state
    std::vector<std::vector<T>> xs(nsteps + 1, std::vector<T>(pos0, pos0 + 3 * n));
    std::vector<uint8_t> moved(n, 1);
    std::vector<int32_t> nnz(n, 0);
    std::vector<double> F(3 * n, 0.0);
    orc_params q = *p;
    for (int32_t s = 0; s < nsteps; ++s) {
        xs[s + 1] = xs[s];
        const int rc = step_impl(n, xs[s + 1].data(), diam, moved.data(), nnz.data(), F.data(), s, &q,
                                 (uint8_t*)nullptr, (double*)nullptr);
        if (rc != 0) return rc;
    }
    const std::vector<T>& xT = xs[nsteps];
    double L = 0.0;
    std::vector<double> lam(3 * n);
    for (int64_t c = 0; c < 3 * n; ++c) {
        const double r = double(xT[c]) - target[c];
        L += r * r;
        lam[c] = 2.0 * r / double(3 * n);
    }
    L /= double(3 * n);
    double gk = 0.0, gg = 0.0;
    for (int32_t s = nsteps - 1; s >= 0; --s) {
        const T* x = xs[s].data();
        Grid<T> g;
        const int rc = build_grid(g, n, x, inv_h, p->order);
        if (rc != 0) return rc;
        const double R2 = R * R;
        // w_i = (dDelta_i/dF_i)^T lambda_i, plus sum_j dF_i/dk, dF_i/dgamma
        std::vector<double> w(3 * n, 0.0);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : gk, gg)
        for (int64_t i = 0; i < n; ++i) {
            const Vec3 xi = load(x, i);
            double Fx = 0, Fy = 0, Fz = 0, Kx = 0, Ky = 0, Kz = 0, Gx = 0, Gy = 0, Gz = 0;
            for_candidates(g, i, [&](int64_t j) {
                const Vec3 xj = load(x, j);
                if (!(sq3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z) < R2)) return;
                const PairTerm pt = pair_term(xi, d[i], xj, d[j], p->k, p->gamma);
                if (!pt.contact) return;
                Fx += pt.fx; Fy += pt.fy; Fz += pt.fz;
                const double ex = xi.x - xj.x, ey = xi.y - xj.y, ez = xi.z - xj.z;
                const double dist = std::sqrt(sq3(ex, ey, ez));
                const double ri = 0.5 * d[i], rj = 0.5 * d[j], S = ri + rj;
                const double delta = S - dist, rho = (ri * rj) / S;
                const double ux = ex / dist, uy = ey / dist, uz = ez / dist;
                Kx += delta * ux; Ky += delta * uy; Kz += delta * uz;            // dF/dk
                const double sr = std::sqrt(rho * delta);
                Gx -= sr * ux; Gy -= sr * uy; Gz -= sr * uz;                      // dF/dgamma
            });
            const double Fn = std::sqrt(sq3(Fx, Fy, Fz));
            if (!(Fn > p->f_adh)) continue;  // below threshold: Delta = 0, no derivative
            const double li[3] = {lam[3 * i], lam[3 * i + 1], lam[3 * i + 2]};
            double wi[3];
            const double mx = p->mu * Fx, my = p->mu * Fy, mz = p->mu * Fz;
            const double un = std::sqrt(sq3(mx, my, mz));
            if (un > p->delta_max) {
                // Delta = delta_max F/|F|: dDelta/dF = delta_max/|F| (I - F^ F^T)
                const double fh[3] = {Fx / Fn, Fy / Fn, Fz / Fn};
                const double dot = li[0] * fh[0] + li[1] * fh[1] + li[2] * fh[2];
                for (int a = 0; a < 3; ++a) wi[a] = p->delta_max / Fn * (li[a] - dot * fh[a]);
            } else {
                for (int a = 0; a < 3; ++a) wi[a] = p->mu * li[a];
            }
            w[3 * i] = wi[0]; w[3 * i + 1] = wi[1]; w[3 * i + 2] = wi[2];
            gk += wi[0] * Kx + wi[1] * Ky + wi[2] * Kz;
            gg += wi[0] * Gx + wi[1] * Gy + wi[2] * Gz;
        }
        // lambda_m <- lambda_m + sum_{j in contact with m} A_mj (w_m - w_j),
        // A = d(phi)/de for phi(e) = g(|e|) e, g(d) = f(S - d)/d.
        std::vector<double> nl(3 * n);
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t m = 0; m < n; ++m) {
            const Vec3 xm = load(x, m);
            double acc[3] = {lam[3 * m], lam[3 * m + 1], lam[3 * m + 2]};
            for_candidates(g, m, [&](int64_t j) {
                const Vec3 xj = load(x, j);
                const double ex = xm.x - xj.x, ey = xm.y - xj.y, ez = xm.z - xj.z;
                const double s2 = sq3(ex, ey, ez);
                if (!(s2 < R2)) return;
                const double ri = 0.5 * d[m], rj = 0.5 * d[j], S = ri + rj;
                if (!(s2 > 0.0) || !(s2 < S * S)) return;
                const double dist = std::sqrt(s2);
                const double delta = S - dist, rho = (ri * rj) / S;
                const double f = p->k * delta - p->gamma * std::sqrt(rho * delta);
                const double fp = p->k - p->gamma * rho / (2.0 * std::sqrt(rho * delta));  // df/ddelta
                const double gd = f / dist;
                const double gprime = -(fp * dist + f) / (dist * dist);                    // dg/dd
                const double e[3] = {ex, ey, ez};
                const double v[3] = {w[3 * m] - w[3 * j], w[3 * m + 1] - w[3 * j + 1], w[3 * m + 2] - w[3 * j + 2]};
                const double ev = e[0] * v[0] + e[1] * v[1] + e[2] * v[2];
                for (int a = 0; a < 3; ++a) acc[a] += gd * v[a] + gprime / dist * e[a] * ev;
            });
            nl[3 * m] = acc[0]; nl[3 * m + 1] = acc[1]; nl[3 * m + 2] = acc[2];
        }
        lam.swap(nl);
    }
    if (posT) std::memcpy(posT, xT.data(), 3 * n * sizeof(T));
    if (loss) *loss = L;
    if (dL_dx0) std::memcpy(dL_dx0, lam.data(), 3 * n * sizeof(double));
    if (dL_dparams) { dL_dparams[0] = gk; dL_dparams[1] = gg; }
    return 0;
}

}  // namespace

extern "C" {

// Section 4.2 step D for a D-dimensional box (D = 2 or 3).  Writes at most cap
// entries and returns the total number of entries.
int64_t orc_gap_table(int32_t D, const int64_t* dims, int64_t* box_counter, int64_t* offset, int64_t cap) {
    if (D < 1 || D > 3) return -1;
    for (int a = 0; a < D; ++a)
        if (dims[a] < 1 || dims[a] > kMaxDim) return -3;
    const GapTable t = build_gap_table(dims, D);
    const int64_t ne = int64_t(t.counter.size());
    for (int64_t e = 0; e < ne && e < cap; ++e) {
        box_counter[e] = t.counter[e];
        offset[e] = t.offset[e];
    }
    return ne;
}

// Ranks of boxes q (n x D coordinates) via the step-D table, and the Morton
// codes of ranks r via step E.  Either output may be null.
int64_t orc_ranks(int32_t D, const int64_t* dims, int64_t n, const int64_t* q, int64_t* rank_out,
                  int64_t nr, const int64_t* ranks, uint64_t* code_out) {
    if (D < 1 || D > 3) return -1;
    const GapTable t = build_gap_table(dims, D);
    for (int64_t i = 0; i < n; ++i) rank_out[i] = rank_of_code(t, morton(&q[D * i], D, t.L));
    for (int64_t i = 0; i < nr; ++i) code_out[i] = code_of_rank(t, ranks[i]);
    return 0;
}

uint64_t orc_morton(int32_t D, const int64_t* q, int32_t levels) { return morton(q, D, levels); }

int64_t orc_grid_f64(int64_t n, const double* pos, double inv_h, int64_t* cmin, int64_t* dims, uint32_t* key,
                     uint32_t* perm, uint32_t* cell_start, int64_t cell_cap, int32_t order) {
    return grid_impl(n, pos, inv_h, cmin, dims, key, perm, cell_start, cell_cap, order);
}
int64_t orc_grid_f32(int64_t n, const float* pos, double inv_h, int64_t* cmin, int64_t* dims, uint32_t* key,
                     uint32_t* perm, uint32_t* cell_start, int64_t cell_cap, int32_t order) {
    return grid_impl(n, pos, inv_h, cmin, dims, key, perm, cell_start, cell_cap, order);
}

// Hilbert index of n points (n x 3 coordinates below 2^b).
int64_t orc_hilbert(int64_t n, const int64_t* q, int32_t b, uint64_t* out) {
    if (b < 0 || b > 21) return -1;
    for (int64_t i = 0; i < n; ++i) out[i] = hilbert_index(&q[3 * i], b);
    return 0;
}

int64_t orc_neighbors_f64(int64_t n, const double* pos, double R, double inv_h, int64_t* start, uint32_t* nbr,
                          int64_t cap) {
    return neighbors_impl(n, pos, R, inv_h, start, nbr, cap);
}
int64_t orc_neighbors_f32(int64_t n, const float* pos, double R, double inv_h, int64_t* start, uint32_t* nbr,
                          int64_t cap) {
    return neighbors_impl(n, pos, R, inv_h, start, nbr, cap);
}

int orc_step_f64(int64_t n, double* pos, const double* diam, uint8_t* moved, int32_t* nnz, double* force,
                 int64_t t, const orc_params* p, uint8_t* is_static, double* disp) {
    return step_impl(n, pos, diam, moved, nnz, force, t, p, is_static, disp);
}
int orc_step_f32(int64_t n, float* pos, const float* diam, uint8_t* moved, int32_t* nnz, double* force,
                 int64_t t, const orc_params* p, uint8_t* is_static, double* disp) {
    return step_impl(n, pos, diam, moved, nnz, force, t, p, is_static, disp);
}

int orc_adjoint_f64(int64_t n, const double* pos0, const double* diam, int32_t nsteps, const orc_params* p,
                    const double* target, double* posT, double* loss, double* dL_dx0, double* dL_dparams) {
    return adjoint_impl(n, pos0, diam, nsteps, p, target, posT, loss, dL_dx0, dL_dparams);
}
int orc_adjoint_f32(int64_t n, const float* pos0, const float* diam, int32_t nsteps, const orc_params* p,
                    const double* target, float* posT, double* loss, double* dL_dx0, double* dL_dparams) {
    return adjoint_impl(n, pos0, diam, nsteps, p, target, posT, loss, dL_dx0, dL_dparams);
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

}  // extern "C"

extern "C" {
int orc_sample_f64(int64_t n, const double* pos, const double* diam, const orc_params* p, int64_t ns,
                   const int64_t* ids, double* F, int32_t* nnz, double* new_pos) {
    return sample_impl(n, pos, diam, p, ns, ids, F, nnz, new_pos);
}
int orc_sample_f32(int64_t n, const float* pos, const float* diam, const orc_params* p, int64_t ns,
                   const int64_t* ids, double* F, int32_t* nnz, float* new_pos) {
    return sample_impl(n, pos, diam, p, ns, ids, F, nnz, new_pos);
}
}  // extern "C"
