// grid_kernels.hip -- uniform-grid build of one step (Section 3.1) with boxes
// in gap-free Morton order (Section 4.2, steps D-F; or the Hilbert order of
// the super-boxes), counted per super-box (the aligned 2x2x2 blocks of
// boxes, whose agents are contiguous in that order):
//   bbox     box extent of the agents (per simulation)
//   setup    dims, box and super-box counts and bases of every simulation;
//            full or update build (several simulations: those whose extent
//            changed are rebuilt inside an update, with a fresh table stamp)
//   keys     super-box key and octant of every agent + histogram (atomics);
//            an update build: only the agents that left their box (all of a
//            rebuilt simulation's), and with the static test the moved
//            octants of every super-box
//   scan     exclusive scan of the super-box counts (tile sums, their scan,
//            rescan); an update build also lists the changed super-boxes
//            and refreshes the table entries of the others
//   scatter  records of the agents of the (re)built super-boxes, in arrival
//            order inside a super-box
//   fixup    canonical (box, id) order inside each (re)built super-box, its
//            agents written to loose slots + the row-major super-box table
#include "force_loop.h"

#include <algorithm>

namespace abm {

// ------------------------------------------------------------------ init
template <class T>
__global__ void k_pack(Buffers<T> b, const T* __restrict__ pos, const T* __restrict__ diam) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    V4<T> p;
    p.x = pos[3 * size_t(i)];
    p.y = pos[3 * size_t(i) + 1];
    p.z = pos[3 * size_t(i) + 2];
    p.w = diam[i];
    const double d = double(p.w);
    if (!(d > 0.0) || !isfinite(d) || !isfinite(double(p.x)) || !isfinite(double(p.y)) || !isfinite(double(p.z)))
        raise_error(b.g, kErrNonfinite);
    pos4_ptr(b, 0)[i] = p;
    b.ids[0][i] = i;
    b.flags[0][i] = kMovedBit;   // step 0 has no history: every agent counts as moved
    if (b.force[0]) {
        b.force[0][3 * size_t(i)] = 0.0;
        b.force[0][3 * size_t(i) + 1] = 0.0;
        b.force[0][3 * size_t(i) + 2] = 0.0;
    }
}

template <class T>
void launch_pack(const Buffers<T>& b, const T* pos, const T* diam, hipStream_t s) {
    const uint32_t blocks = (b.n + 255) / 256;
    hipLaunchKernelGGL(k_pack<T>, dim3(blocks), dim3(256), 0, s, b, pos, diam);
}

// Occupied boxes of one simulation's initial grid (lower box lo, dims d):
// one bit per box, set by the agents in it, then counted.  The mean number
// of agents per occupied box chooses the neighbour walk's width at init
// (clustered agents fill few boxes of a large extent densely).
template <class T>
__global__ void k_mark_boxes(Buffers<T> b, int32_t lo0, int32_t lo1, int32_t lo2, uint32_t d0, uint32_t d1,
                             uint32_t d2, uint32_t* __restrict__ bits) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const V4<T> p = pos4_ptr(b, 0)[i];
    const double inv_h = b.sims[0].inv_h;
    int32_t c[3];
    if (!(box_coord(double(p.x), inv_h, &c[0]) && box_coord(double(p.y), inv_h, &c[1]) &&
          box_coord(double(p.z), inv_h, &c[2])))
        return;
    const int64_t q0 = int64_t(c[0]) - lo0, q1 = int64_t(c[1]) - lo1, q2 = int64_t(c[2]) - lo2;
    if (q0 < 0 || q1 < 0 || q2 < 0 || q0 >= int64_t(d0) || q1 >= int64_t(d1) || q2 >= int64_t(d2)) return;
    const uint64_t lin = (uint64_t(q2) * d1 + uint64_t(q1)) * d0 + uint64_t(q0);
    atomicOr(&bits[lin >> 5], 1u << (lin & 31u));
}

__global__ void k_count_bits(const uint32_t* __restrict__ bits, uint64_t nwords, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_sum;
    if (threadIdx.x == 0) s_sum = 0ull;
    __syncthreads();
    unsigned long long t = 0;
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nwords; w += uint64_t(gridDim.x) * blockDim.x)
        t += uint64_t(__popc(bits[w]));
    for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
    if (lane_id() == 0) atomicAdd(&s_sum, t);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd(out, s_sum);
}

__global__ void k_zero_words(uint32_t* __restrict__ p, uint64_t n, unsigned long long* __restrict__ out) {
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < n; w += uint64_t(gridDim.x) * blockDim.x)
        p[w] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = 0ull;
}

template <class T>
void launch_occupied_boxes(const Buffers<T>& b, const int32_t lo[3], const uint32_t dims[3], uint32_t* bits,
                           uint64_t nwords, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_words, dim3(2048), dim3(256), 0, s, bits, nwords, out);
    hipLaunchKernelGGL(k_mark_boxes<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, lo[0], lo[1], lo[2], dims[0],
                       dims[1], dims[2], bits);
    hipLaunchKernelGGL(k_count_bits, dim3(2048), dim3(256), 0, s, bits, nwords, out);
}

// Largest diameter per simulation, as the bits of a positive double (which
// order like unsigned integers).
template <class T>
__global__ void k_radius(Buffers<T> b, int cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = i < b.n;
    int sim = 0;
    unsigned long long v = 0;
    if (active) {
        sim = sim_index(b, i);
        const double d = fabs(double(pos4_ptr(b, cur)[i].w));   // the sign of d is the moved flag
        active = d > 0.0 && isfinite(d);
        v = (unsigned long long)__double_as_longlong(d);
    }
    max_fold_block(sim, active, v, [&](int s) { return &b.sims[s].radius_bits; });
}

template <class T>
void launch_radius(const Buffers<T>& b, int pos_cur, hipStream_t s) {
    const uint32_t blocks = (b.n + 255) / 256;
    hipLaunchKernelGGL(k_radius<T>, dim3(blocks), dim3(256), 0, s, b, pos_cur);
}

// R = the requested interaction radius, or the largest diameter; box edge
// h = cell_factor * R; inv_h = 1 / h and R^2, all in double.
__global__ void k_finish_radius(SimGrid* sims, int nsims) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsims) return;
    SimGrid& G = sims[s];
    const double R = G.radius > 0.0 ? G.radius : __longlong_as_double((long long)G.radius_bits);
    G.radius = R;
    const double cf = G.cell_factor >= 1.0 ? G.cell_factor : 1.0;
    G.inv_h = 1.0 / (R * cf);
    G.r2 = R * R;
}

template <class T>
void launch_finish_radius(const Buffers<T>& b, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_radius, dim3((b.nsims + 255) / 256), dim3(256), 0, s, b.sims, b.nsims);
}

// Extent of caller-layout positions (n x 3 + diameters) for sizing a grid:
// largest diameter, then box coordinates into SimGrid::bbox[0].  Threads loop
// over the agents (a grid of at most kExtentBlocks blocks), so that one
// accumulator takes few same-address atomics.
constexpr uint32_t kExtentBlocks = 1024;
template <class T>
__global__ void k_extent_radius(const T* __restrict__ diam, uint32_t n, Globals* g, SimGrid* sim) {
    bool active = false;
    unsigned long long v = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = double(diam[i]);
        if (!(d > 0.0) || !isfinite(d)) {
            raise_error(g, kErrNonfinite);
            continue;
        }
        const unsigned long long x = (unsigned long long)__double_as_longlong(d);
        v = active && v > x ? v : x;
        active = true;
    }
    max_fold_block(0, active, v, [&](int) { return &sim->radius_bits; });
}

__global__ void k_extent_reset(SimGrid* sim) {
    for (int a = 0; a < 3; ++a) {
        sim->bbox[0][a] = INT32_MAX;
        sim->bbox[0][3 + a] = INT32_MIN;
    }
}

template <class T>
__global__ void k_extent_bbox(const T* __restrict__ pos, uint32_t n, Globals* g, SimGrid* sim) {
    bool active = false;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    const double ih = sim->inv_h;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int32_t c[3];
        const bool ok = box_coord(double(pos[3 * size_t(i)]), ih, &c[0]) &&
                        box_coord(double(pos[3 * size_t(i) + 1]), ih, &c[1]) &&
                        box_coord(double(pos[3 * size_t(i) + 2]), ih, &c[2]);
        if (!ok) {
            raise_error(g, kErrNonfinite);
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], c[a]);
            hi[a] = max(hi[a], c[a]);
        }
        active = true;
    }
    bbox_fold_block(0, active, lo, hi, [&](int) { return sim->bbox[0]; });
}

template <class T>
void launch_extent(const T* pos, const T* diam, uint32_t n, Globals* g, SimGrid* sim, hipStream_t s) {
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, kExtentBlocks);
    hipLaunchKernelGGL(k_extent_radius<T>, dim3(blocks), dim3(256), 0, s, diam, n, g, sim);
    hipLaunchKernelGGL(k_finish_radius, dim3(1), dim3(64), 0, s, sim, 1);
    hipLaunchKernelGGL(k_extent_reset, dim3(1), dim3(1), 0, s, sim);
    hipLaunchKernelGGL(k_extent_bbox<T>, dim3(blocks), dim3(256), 0, s, pos, n, g, sim);
}

// A parameter change counts as a move of every agent (Section 5: a changed
// attribute that can change the force unsets static agents).
template <class T>
__global__ void k_mark_moved(Buffers<T> b, int cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.n) b.flags[cur][i] |= kMovedBit;
}

template <class T>
void launch_mark_moved(const Buffers<T>& b, int pos_cur, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_moved<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, pos_cur);
}

__global__ void k_set_params(SimGrid* sims, int nsims, double k, double gamma, double mu, double f_adh,
                             double delta_max) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsims) return;
    sims[s].k = k;
    sims[s].gamma = gamma;
    sims[s].mu = mu;
    sims[s].f_adh = f_adh;
    sims[s].delta_max = delta_max;
}

void launch_set_params(SimGrid* sims, int nsims, double k, double gamma, double mu, double f_adh, double delta_max,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_set_params, dim3((nsims + 255) / 256), dim3(256), 0, s, sims, nsims, k, gamma, mu, f_adh,
                       delta_max);
}

// Set every replica of one bbox slot to the empty box.
__global__ void k_reset_bbox(int32_t* rep, int nsims, int slot) {
    const size_t per = size_t(kReplicas) * size_t(nsims);
    const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= per) return;
    int32_t* t = rep + (size_t(slot) * per + e) * 6;
    for (int a = 0; a < 3; ++a) {
        t[a] = INT32_MAX;
        t[3 + a] = INT32_MIN;
    }
}

template <class T>
void launch_reset_bbox(const Buffers<T>& b, int parity, hipStream_t s) {
    const uint32_t per = uint32_t(kReplicas) * uint32_t(b.nsims);
    hipLaunchKernelGGL(k_reset_bbox, dim3((per + 255) / 256), dim3(256), 0, s, b.bbox_rep, b.nsims, parity);
}

template <class T>
__global__ void k_bbox(Buffers<T> b, int cur, int slot) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = i < b.n;
    int sim = 0;
    int32_t c[3] = {0, 0, 0};
    if (active) {
        sim = sim_index(b, i);
        const V4<T> p = pos4_ptr(b, cur)[i];
        const double ih = b.sims[sim].inv_h;
        const bool ok = box_coord(double(p.x), ih, &c[0]) && box_coord(double(p.y), ih, &c[1]) &&
                        box_coord(double(p.z), ih, &c[2]);
        if (!ok) {
            raise_error(b.g, kErrNonfinite);
            active = false;
        }
    }
    bbox_fold_block(sim, active, c, [&](int s) { return bbox_replica(b, slot, s); });
}

template <class T>
void launch_bbox(const Buffers<T>& b, int pos_cur, int parity, hipStream_t s) {
    launch_reset_bbox<T>(b, parity, s);
    const uint32_t blocks = (b.n + 255) / 256;
    hipLaunchKernelGGL(k_bbox<T>, dim3(blocks), dim3(256), 0, s, b, pos_cur, parity);
}

// ------------------------------------------------------------------ setup
// One block: per simulation, dims and box count from its bbox accumulator,
// then an exclusive scan of the box counts gives each simulation's base in
// the shared box arrays.  Also clears the other accumulator for this step's
// move kernel and the step statistics.
constexpr int kSetupThreads = 1024;
constexpr int kSetupLdsSims = 512;   // simulations whose box ranges the block folds in LDS
constexpr uint32_t kFixupLanes = 8;   // threads per changed super-box in an update build

__global__ __launch_bounds__(kSetupThreads) void k_setup(Globals* g, SimGrid* sims, int32_t* rep, int nsims,
                                                           int parity, uint32_t super_capacity, int allow_inc,
                                                           uint32_t n) {
    __shared__ unsigned long long s_wave[kSetupThreads / 64];
    __shared__ unsigned long long s_carry;
    __shared__ uint32_t s_same;
    __shared__ uint32_t s_flags;   // the decision: update build (bit 0), the current stamp
    __shared__ uint32_t s_moving;  // agents of the simulations whose grid changed
    __shared__ uint32_t s_nchanged;   // ... and their number
    __shared__ int32_t s_bb[kSetupLdsSims][6];
    if (threadIdx.x == 0) {
        s_carry = 0;
        s_same = 1u;
        s_moving = 0u;
        s_nchanged = 0u;
    }
    // each simulation's box range from its replicas: one wave per simulation,
    // one lane per replica (below kSetupLdsSims simulations; else per thread)
    static_assert(kReplicas == 64, "one lane per replica");
    const bool wave_fold = nsims <= kSetupLdsSims;
    if (wave_fold) {
        for (int s = int(threadIdx.x >> 6); s < nsims; s += kSetupThreads / 64) {
            const int32_t* t = rep + ((size_t(parity) * kReplicas + size_t(lane_id())) * size_t(nsims) + s) * 6;
            int32_t bb[6];
            for (int a = 0; a < 6; ++a) bb[a] = t[a];
            for (int a = 0; a < 3; ++a) {
                bb[a] = wave_min(bb[a]);
                bb[3 + a] = wave_max(bb[3 + a]);
            }
            if (lane_id() == 0)
                for (int a = 0; a < 6; ++a) s_bb[s][a] = bb[a];
        }
    }
    // the other accumulator slot and this step's statistics start empty
    const size_t per = size_t(kReplicas) * size_t(nsims);
    for (size_t e = threadIdx.x; e < per; e += kSetupThreads) {
        int32_t* t = rep + (size_t(parity ^ 1) * per + e) * 6;
        for (int a = 0; a < 3; ++a) {
            t[a] = INT32_MAX;
            t[3 + a] = INT32_MIN;
        }
    }
    for (int e = int(threadIdx.x); e < kReplicas * 2; e += kSetupThreads) g->stats[parity][e >> 1][e & 1] = 0ull;
    for (int e = int(threadIdx.x); e < kReplicas * 3; e += kSetupThreads) g->fsum[parity][e / 3][e % 3] = 0.0;
    for (int e = int(threadIdx.x); e < kReplicas; e += kSetupThreads) g->dmax[parity][e] = 0ull;
    __syncthreads();
    bool t_all_valid = true, t_some_same = false;   // over this thread's simulations
    for (int chunk = 0; chunk < nsims; chunk += kSetupThreads) {
        const int s = chunk + int(threadIdx.x);
        uint32_t nb = 0, nsup = 0;
        bool same = true, last_valid = true;
        if (s < nsims) {
            SimGrid& G = sims[s];
            last_valid = G.valid != 0u;
            same = last_valid;   // the last grid of this simulation was built
            int32_t bb[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
            if (wave_fold) {
                for (int a = 0; a < 6; ++a) bb[a] = s_bb[s][a];
            } else {
                for (int r = 0; r < kReplicas; ++r) {
                    const int32_t* t = rep + ((size_t(parity) * kReplicas + r) * size_t(nsims) + s) * 6;
                    for (int a = 0; a < 3; ++a) {
                        bb[a] = min(bb[a], t[a]);
                        bb[3 + a] = max(bb[3 + a], t[3 + a]);
                    }
                }
            }
            bool ok = true;
            uint64_t total = 1;
            int levels = 0;
            for (int a = 0; a < 3; ++a) {
                const int64_t lo = bb[a], hi = bb[3 + a];
                const int64_t d = hi - lo + 1;
                if (hi < lo || d > int64_t(kMaxBoxesPerAxis)) ok = false;
                const uint32_t du = ok ? uint32_t(d) : 1u;
                same = same && G.cmin[a] == int32_t(lo) && G.dims[a] == du;
                G.cmin[a] = int32_t(lo);
                G.dims[a] = du;
                total *= du;
                while ((1u << levels) < du) ++levels;
            }
            if (total > uint64_t(G.cap) || total >= (uint64_t(1) << 32)) ok = false;
            G.levels = levels;
            G.valid = ok ? 1u : 0u;
            G.nboxes = ok ? uint32_t(total) : 0u;
            uint32_t ns = 1;
            for (int a = 0; a < 3; ++a) {
                const uint32_t sd = ok ? super_dim(G.dims[a]) : 1u;
                G.sdims[a] = sd;
                ns *= sd;
            }
            G.slevels = levels > 0 ? levels - 1 : 0;
            if (ok && nsims > 1 && ns > G.scap) {   // beyond this simulation's table range
                ok = false;
                G.valid = 0u;
                G.nboxes = 0u;
            }
            G.nsuper = ok ? ns : 0u;
            nb = G.nboxes;
            nsup = G.nsuper;
            same = same && ok;
            if (!ok) raise_error(g, kErrGrid);
            t_all_valid = t_all_valid && last_valid && ok;
            t_some_same = t_some_same || same;
            G.rebuild = same ? 0u : 1u;   // provisional: the grid changed
            if (!same) {
                atomicAdd(&s_moving, G.agent_end - G.agent_begin);
                atomicAdd(&s_nchanged, 1u);
            }
        }
        if (!__syncthreads_and(same ? 1 : 0) && threadIdx.x == 0) s_same = 0u;
        // block exclusive scans of nb (box bases) and nsup (super-box bases)
        unsigned long long x = (unsigned long long)nb | ((unsigned long long)nsup << 32);
        const int lane = int(threadIdx.x & 63u), wave = int(threadIdx.x >> 6);
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) s_wave[wave] = x;
        __syncthreads();
        unsigned long long wave_off = 0;
        for (int w = 0; w < wave; ++w) wave_off += s_wave[w];
        const unsigned long long own = (unsigned long long)nb | ((unsigned long long)nsup << 32);
        const unsigned long long off = wave_off + x - own;
        const unsigned long long bbase = (s_carry & 0xFFFFFFFFull) + (off & 0xFFFFFFFFull);
        const unsigned long long sbase = (s_carry >> 32) + (off >> 32);
        if (s < nsims) {
            sims[s].box_base = uint32_t(bbase);
            if (nsims == 1) sims[s].sbase = uint32_t(sbase);   // several: fixed ranges
        }
        __syncthreads();
        // box counts are bounded by the capacities, whose sum fits 32 bits,
        // so neither half of the packed sums carries into the other
        if (threadIdx.x == kSetupThreads - 1) s_carry = ((bbase + nb) & 0xFFFFFFFFull) | ((sbase + nsup) << 32);
        __syncthreads();
    }
    const bool all_valid = __syncthreads_and(t_all_valid ? 1 : 0) != 0;
    const bool some_same = __syncthreads_or(t_some_same ? 1 : 0) != 0;
    if (threadIdx.x == 0) {
        // one simulation: its super-boxes; several: every table range, fixed
        unsigned long long total = nsims == 1 ? s_carry >> 32 : (unsigned long long)super_capacity;
        if (total > super_capacity || total >= kMaxSuperBoxes) {
            raise_error(g, kErrGrid);
            total = 0;
            for (int s = 0; s < nsims; ++s) sims[s].valid = 0;
        }
        g->total_super = uint32_t(total);
        // An update of the last grid needs the agents stored in that grid's
        // canonical order (the caller's allow_inc).  One simulation: the same
        // boxes (extent).  Several: every simulation's last and new grid
        // valid, and some simulation with its extent kept; the others are
        // rebuilt inside the update (all their agents move to their new keys).
        // Rebuilding simulations inside an update moves all their agents
        // through the movers' path, whose arrival counters serialise runs of
        // agents bound for one super-box: with a quarter of the agents or
        // more in changed simulations, a full build is the faster one.
        const bool inc = allow_inc && total > 0 &&
                         (nsims == 1 ? s_same != 0u : all_valid && some_same && 4ull * s_moving < n);
        g->inc = inc ? 1u : 0u;
        g->epoch = g->epoch + 1u ? g->epoch + 1u : 1u;
        g->ndirty = 0u;
        g->napp = n;   // a full build fills the whole append region (an update: set by its scan)
        // A full build marks every simulation's table entries with a fresh
        // stamp (the host clears the table before the 15-bit stamp wraps); an
        // update keeps the entries of the super-boxes it does not rebuild, and
        // the simulations rebuilt inside it take a fresh stamp
        const bool rebuilds = inc && nsims > 1 && s_same == 0u;
        g->rebuilt = rebuilds ? s_nchanged : 0u;
        if (!inc || rebuilds) g->stamp = g->stamp + 1;
        s_flags = (inc ? 1u : 0u) | (g->stamp << 1);
    }
    __syncthreads();
    const bool inc = (s_flags & 1u) != 0u;
    const uint32_t stamp = s_flags >> 1;
    for (int s = int(threadIdx.x); s < nsims; s += kSetupThreads) {
        SimGrid& G = sims[s];
        const bool rb = inc && nsims > 1 && G.rebuild != 0u;
        G.rebuild = rb ? 1u : 0u;
        if (!inc || rb) G.stamp = stamp;
    }
}

template <class T>
void launch_setup(const Buffers<T>& b, int parity, bool allow_inc, hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(kSetupThreads), 0, s, b.g, b.sims, b.bbox_rep, b.nsims, parity,
                       b.super_capacity, allow_inc ? 1 : 0, b.n);
}

// ------------------------------------------------------------------ keys
// Key of a position: (global super-box rank << 3) | octant of its box (x bit
// lowest).  The super-box rank is gap-free over the super grid: in Morton
// order from the closed-form walk of gapfree_rank, in Hilbert order from the
// walk down the curve's octree (hil: the curve's tables, an LDS copy).
// false if the position lies outside the grid.
template <class T>
__device__ __forceinline__ bool super_key(const SimGrid& G, const V4<T>& p, uint32_t* key, const HilbertTables* hil) {
    uint32_t q[3];
    if (!box_of<T>(G, p, q)) return false;
    uint32_t rank;
    if (hil) {
        rank = hilbert_rank(q[0] >> 1, q[1] >> 1, q[2] >> 1, G.sdims[0], G.sdims[1], G.sdims[2], G.slevels, 1u,
                            hil->before, hil->next);
    } else {
        rank = gapfree_rank(q[0] >> 1, q[1] >> 1, q[2] >> 1, G.sdims[0], G.sdims[1], G.sdims[2], G.slevels);
    }
    *key = ((G.sbase + rank) << 3) | (q[0] & 1u) | ((q[1] & 1u) << 1) | ((q[2] & 1u) << 2);
    return true;
}

// Lanes of a wave that hold equal values of k come in runs (agents of one
// super-box are neighbours in storage).  wave_run_add adds each run's length
// to arr[k] (subtracts it with `subtract`) with one atomic and returns every
// lane's index in arr[k]'s count (an add).
__device__ __forceinline__ uint32_t wave_run_add(uint32_t* arr, bool act, uint32_t k, bool subtract = false) {
    const int lane = lane_id();
    const uint32_t pk = __shfl_up(k, 1, 64);
    const int pact = __shfl_up(act ? 1 : 0, 1, 64);
    const bool head = act && (lane == 0 || !pact || pk != k);
    const unsigned long long heads = __ballot(head);
    const unsigned long long brk = __ballot(!act || head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane
    const int leader = act ? 63 - __clzll((long long)(heads & upto)) : lane;
    const unsigned long long above = brk & ~upto;
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    uint32_t old = 0;
    if (head) old = atomicAdd(&arr[k], subtract ? 0u - uint32_t(next - lane) : uint32_t(next - lane));
    old = __shfl(old, leader, 64);
    return old + uint32_t(lane - leader);
}

// The same runs for a bit mask: each run's OR goes to arr[k] with one
// atomicOr (a lane with act false is in no run).
__device__ __forceinline__ void wave_run_or(uint32_t* arr, bool act, uint32_t k, uint32_t bits) {
    const int lane = lane_id();
    const uint32_t kk = act ? k : 0xFFFFFFFFu;
    uint32_t acc = act ? bits : 0u;
    // lane l gathers the run from l on: after the step of width d it holds
    // lanes [l, l + 2d) of its run
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_down(acc, d, 64);
        const uint32_t ok = __shfl_down(kk, d, 64);
        if (lane + d < 64 && ok == kk) acc |= o;
    }
    const uint32_t pk = __shfl_up(kk, 1, 64);
    if (act && (lane == 0 || pk != kk) && acc) atomicOr(&arr[k], acc);
}

// Full build: key of every agent and its arrival index in its super-box
// (histogram atomics).  Update build (the last grid's extent, agents stored in
// its canonical order): only agents that left their box get a new key; each
// that enters another super-box moves one count from its old to its new
// super-box and marks both as changed (the epoch of this build).  All are
// listed in their block's segment, sub[i] noting the ones that moved on.
// With moved_bits, an update build also ORs every agent's moved bit into its
// (last) super-box's mask at its octant; the scan moves the masks of the kept
// super-boxes into their table entries (a rebuilt one gets its bits from the
// fix-up).  A block covers kKeysPer runs of kKeysThreads consecutive agents;
// in an update build a thread requests the flags of its kKeysPer agents
// together.
constexpr int kKeysThreads = 256;
constexpr int kKeysPer = 4;
constexpr uint32_t kKeysSpan = kKeysThreads * kKeysPer;
template <class T>
__global__ __launch_bounds__(kKeysThreads) void k_keys(Buffers<T> b, int cur, int moved_bits) {
    __shared__ uint32_t s_movers;
    __shared__ uint32_t s_list[kKeysSpan];
    __shared__ __align__(16) HilbertTables s_hil;
    const uint32_t i0 = blockIdx.x * kKeysSpan + threadIdx.x;
    const HilbertTables* hil = nullptr;
    if (b.hil) {   // the same for the whole block
        const uint32_t* src = reinterpret_cast<const uint32_t*>(b.hil);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s_hil);
        for (uint32_t w = threadIdx.x; w < uint32_t(sizeof(HilbertTables) / 4); w += kKeysThreads) dst[w] = src[w];
        __syncthreads();
        hil = &s_hil;
    }
    if (!b.g->inc) {
#pragma unroll
        for (int k = 0; k < kKeysPer; ++k) {
            const uint32_t i = i0 + uint32_t(k) * kKeysThreads;
            bool act = false;
            uint32_t key = 0;
            if (i < b.n) {
                const SimGrid& G = b.sims[sim_index(b, i)];
                if (G.valid) {
                    if (super_key<T>(G, pos4_ptr(b, cur)[i], &key, hil)) {
                        act = true;
                    } else {   // the extent is computed from these very positions
                        raise_error(b.g, kErrInternal);
                        key = 0xFFFFFFFFu;
                    }
                    b.key[i] = key;
                }
            }
            const uint32_t sub = wave_run_add(b.count, act, key >> 3);
            if (act) b.sub[i] = sub;
        }
        return;
    }
    // flags and (for the moved octants) keys requested together
    uint32_t f[kKeysPer], sk[kKeysPer];
#pragma unroll
    for (int k = 0; k < kKeysPer; ++k) {
        const uint32_t i = i0 + uint32_t(k) * kKeysThreads;
        f[k] = i < b.n ? b.flags[cur][i] : 0u;
        sk[k] = moved_bits && i < b.n ? b.skey[cur][i] : kDeadKey;
    }
    // several simulations: every agent of a simulation rebuilt inside this
    // update counts as having left its box (also for the scatter, which reads
    // the flag again)
    if (b.sim_of) {
#pragma unroll
        for (int k = 0; k < kKeysPer; ++k) {
            const uint32_t i = i0 + uint32_t(k) * kKeysThreads;
            if (i < b.n && !(f[k] & kBoxChangedBit) && b.sims[sim_index(b, i)].rebuild) {
                f[k] |= kBoxChangedBit;
                b.flags[cur][i] = f[k];
            }
        }
    }
    if (moved_bits) {   // agents in storage order: equal super-boxes in runs
        const uint32_t total = b.g->total_super;
#pragma unroll
        for (int k = 0; k < kKeysPer; ++k) {
            const uint32_t key = sk[k];
            const bool act = key != kDeadKey && (key >> 3) < total;
            wave_run_or(b.mmask, act, key >> 3, (f[k] & kMovedBit) << (key & 7u));
        }
    }
    // the block's agents that left their box, gathered in LDS, then taken
    // one per thread, so that their dependent loads overlap
    if (threadIdx.x == 0) s_movers = 0u;
    __syncthreads();
    for (int k = 0; k < kKeysPer; ++k)
        if (f[k] & kBoxChangedBit) s_list[atomicAdd(&s_movers, 1u)] = i0 + uint32_t(k) * kKeysThreads;
    __syncthreads();
    // the count moves as runs of equal keys, one atomic per run (a simulation
    // rebuilt inside the update moves runs of agents of one super-box)
    const uint32_t nl = s_movers, ep = b.g->epoch, total = b.g->total_super;
    for (uint32_t j0 = 0; j0 < nl; j0 += kKeysThreads) {
        const uint32_t j = j0 + threadIdx.x;
        const bool in = j < nl;
        const uint32_t i = in ? s_list[j] : 0u;
        uint32_t old = 0, key = 0, real = 0;
        bool rb = false;
        if (in) {
            const SimGrid& G = b.sims[sim_index(b, i)];
            old = b.skey[cur][i];
            key = old;
            if (!G.valid || (old >> 3) >= total || !super_key<T>(G, pos4_ptr(b, cur)[i], &key, hil)) {
                raise_error(b.g, kErrInternal);
                key = old;
            } else {
                real = key != old ? 1u : 0u;
                rb = G.rebuild != 0u;
            }
        }
        (void)wave_run_add(b.count, real != 0u, old >> 3, true);
        (void)wave_run_add(b.count, real != 0u, key >> 3);
        if (in) {
            // a rebuilt simulation's super-boxes are all rebuilt: the same
            // key names another block of boxes in its new grid
            if (real || rb) {
                b.dirty[old >> 3] = ep;
                b.dirty[key >> 3] = ep;
            }
            b.key[i] = key;   // read by the scatter for every agent that left its box
            b.sub[i] = real;  // ... and whether it entered another super-box
            b.movers[blockIdx.x * kKeysSpan + j] = i;
        }
    }
    if (threadIdx.x == 0) b.mcount[blockIdx.x] = nl;
}

// ------------------------------------------------------------------ scan
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t x) {
    const int lane = lane_id();
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of the super-box counts into cell_start[0, total], zeroing
// count, in three passes over tiles of kScanTile super-boxes: per-tile sums,
// a one-block scan of the tile sums, and a per-tile rescan that adds the
// tile's prefix (with few tiles, the rescan adds up the sums before its tile
// itself, and the one-block scan has nothing to do).  Global loads and stores of the counts are striped across
// the block and transposed through LDS, so every wave touches whole cache
// lines.  An update build scans two more quantities along: the changed
// super-boxes (marked with this build's epoch) and their agents; the rescan
// lists the changed super-boxes in rank order, each with its first slot in
// the append region.
__device__ __forceinline__ uint32_t lds_pad(uint32_t i) { return i + (i >> 5); }

// Load tile `tile` of the counts into LDS (striped: thread x takes 4
// consecutive super-boxes per round, with 16-byte loads), return this
// thread's blocked 16 values.  In an update build the counts are the last
// grid's (differences of its starts) plus the changes in `count`, and bit k of
// *dm says that value k's super-box changed; with `refresh` the table entry
// of every other non-empty super-box gets its new first loose slot, its start
// in the storage order (the last grid's start).
struct ScanIn {
    const uint32_t* count;
    const uint32_t* cs_old;
    const uint32_t* dirty;
    const uint32_t* tabidx;
    uint32_t* mmask;
    uint4* cellinfo;
};
constexpr uint32_t kDirtyFlag = 0x80000000u;   // counts stay below 2^31
__device__ __forceinline__ void load_tile(const ScanIn& in, uint32_t ep, bool inc, bool refresh, uint32_t base,
                                          uint32_t total, uint32_t* s_data, uint32_t v[kScanItems], uint32_t* dm) {
    for (int k = 0; k < kScanItems / 4; ++k) {
        const uint32_t e4 = uint32_t(k) * kScanThreads + threadIdx.x;
        const uint32_t g0 = base + 4 * e4;
        uint32_t c4[4] = {0u, 0u, 0u, 0u};
        const bool whole = g0 + 4 <= total;
        if (whole) {
            const uint4 u = reinterpret_cast<const uint4*>(in.count)[g0 >> 2];
            c4[0] = u.x; c4[1] = u.y; c4[2] = u.z; c4[3] = u.w;
        } else {
            for (int c = 0; c < 4; ++c) c4[c] = g0 + c < total ? in.count[g0 + c] : 0u;
        }
        if (inc && g0 < total) {
            uint32_t o[5], d[4], ti[4], mm[4] = {0u, 0u, 0u, 0u};
            if (whole) {
                const uint4 uo = reinterpret_cast<const uint4*>(in.cs_old)[g0 >> 2];
                const uint4 ud = reinterpret_cast<const uint4*>(in.dirty)[g0 >> 2];
                o[0] = uo.x; o[1] = uo.y; o[2] = uo.z; o[3] = uo.w;
                d[0] = ud.x; d[1] = ud.y; d[2] = ud.z; d[3] = ud.w;
                o[4] = in.cs_old[g0 + 4];
                if (refresh) {
                    const uint4 ut = reinterpret_cast<const uint4*>(in.tabidx)[g0 >> 2];
                    ti[0] = ut.x; ti[1] = ut.y; ti[2] = ut.z; ti[3] = ut.w;
                    const uint4 um = reinterpret_cast<const uint4*>(in.mmask)[g0 >> 2];
                    mm[0] = um.x; mm[1] = um.y; mm[2] = um.z; mm[3] = um.w;
                    if (um.x | um.y | um.z | um.w) reinterpret_cast<uint4*>(in.mmask)[g0 >> 2] = make_uint4(0u, 0u, 0u, 0u);
                }
            } else {
                for (int c = 0; c < 4; ++c) {
                    const bool ok = g0 + c < total;
                    o[c] = ok ? in.cs_old[g0 + c] : 0u;
                    d[c] = ok ? in.dirty[g0 + c] : 0u;
                    ti[c] = ok && refresh ? in.tabidx[g0 + c] : 0u;
                    mm[c] = ok && refresh ? in.mmask[g0 + c] : 0u;
                    if (mm[c]) in.mmask[g0 + c] = 0u;
                }
                o[4] = 0u;
                for (int c = 0; c < 4; ++c)
                    if (g0 + c < total) o[c + 1] = in.cs_old[g0 + c + 1];
            }
            for (int c = 0; c < 4; ++c) {
                if (g0 + c >= total) break;
                const bool changed = d[c] == ep;
                c4[c] += o[c + 1] - o[c];
                if (changed) c4[c] |= kDirtyFlag;
                if (refresh && !changed && o[c + 1] != o[c]) {   // first slot, count and moved octants
                    if (ti[c] < total)
                        *reinterpret_cast<uint2*>(&in.cellinfo[ti[c]]) = make_uint2(o[c], (o[c + 1] - o[c]) | (mm[c] << 24));
                }
            }
        }
        for (int c = 0; c < 4; ++c) s_data[lds_pad(4 * e4 + c)] = c4[c];
    }
    __syncthreads();
    *dm = 0u;
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t x = s_data[lds_pad(threadIdx.x * kScanItems + k)];
        v[k] = x & ~kDirtyFlag;
        *dm |= (x >> 31) << k;
    }
}

// This thread's sums: agents, changed super-boxes, agents of changed super-boxes.
__device__ __forceinline__ void thread_sums(const uint32_t v[kScanItems], uint32_t dm, uint32_t x[3]) {
    x[0] = 0u;
    x[2] = 0u;
    for (int k = 0; k < kScanItems; ++k) {
        x[0] += v[k];
        x[2] += ((dm >> k) & 1u) ? v[k] : 0u;
    }
    x[1] = uint32_t(__popc(dm));
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Globals* g, ScanIn in, uint32_t* __restrict__ sums,
                                                               uint32_t ntiles) {
    __shared__ uint32_t s_data[kScanTile + kScanTile / 32];
    __shared__ uint32_t s_wave[3][kScanThreads / 64];
    const uint32_t total = g->total_super;
    const uint32_t tile = blockIdx.x;
    if (tile * uint32_t(kScanTile) >= total || tile >= ntiles) return;
    const bool inc = g->inc != 0u;
    uint32_t v[kScanItems], dm;
    load_tile(in, g->epoch, inc, true, tile * kScanTile, total, s_data, v, &dm);
    uint32_t x[3];
    thread_sums(v, dm, x);
    for (int c = 0; c < 3; ++c) {
        for (int d = 32; d >= 1; d >>= 1) x[c] += __shfl_xor(x[c], d, 64);
        if (lane_id() == 0) s_wave[c][threadIdx.x >> 6] = x[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += s_wave[threadIdx.x][w];
        sums[threadIdx.x * ntiles + tile] = t;
    }
}

// One block: exclusive scan of the tile sums in place; cell_start[total] =
// agents, and in an update build the number of changed super-boxes and of
// their agents.
constexpr int kTileScanThreads = 1024;
// Up to this many tiles in use, the rescan adds up the tile sums before its
// tile itself (at most 24 KB of reads per block) and the one-block scan
// returns at once.
constexpr uint32_t kFusedScanTiles = 2048;
__global__ __launch_bounds__(kTileScanThreads) void k_scan_tiles(Globals* g, uint32_t* __restrict__ sums,
                                                                  uint32_t* __restrict__ cell_start,
                                                                  uint32_t ntiles) {
    __shared__ uint32_t s_wave[kTileScanThreads / 64];
    __shared__ uint32_t s_carry;
    const uint32_t total = g->total_super;
    const uint32_t needed = (total + kScanTile - 1) / kScanTile;
    if (needed <= kFusedScanTiles) return;   // the rescan adds up the tile sums itself
    if (needed > ntiles) {
        if (threadIdx.x == 0) raise_error(g, kErrInternal);
        return;
    }
    const int ncomp = g->inc ? 3 : 1;
    for (int c = 0; c < ncomp; ++c) {
        uint32_t* ts = sums + size_t(c) * ntiles;
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (uint32_t base = 0; base < needed; base += kTileScanThreads) {
            const uint32_t i = base + threadIdx.x;
            const uint32_t x = i < needed ? ts[i] : 0u;
            const uint32_t incl = wave_inclusive(x);
            const int wave = int(threadIdx.x >> 6);
            if (lane_id() == 63) s_wave[wave] = incl;
            __syncthreads();
            uint32_t off = s_carry;
            for (int w = 0; w < wave; ++w) off += s_wave[w];
            if (i < needed) ts[i] = off + incl - x;
            __syncthreads();
            if (threadIdx.x == kTileScanThreads - 1) s_carry = off + incl;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (c == 0 && total > 0) cell_start[total] = s_carry;
            if (c == 1) g->ndirty = s_carry;
            if (c == 2) g->napp = s_carry;
        }
        __syncthreads();
    }
}

// With few tiles (fused), the tile sums are as the first pass wrote them:
// each block adds up those of the tiles before its own (so the one-block scan
// is not launched), and the block of the last tile writes the totals.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Globals* g, ScanIn in, uint32_t* __restrict__ count,
                                                             uint32_t* __restrict__ cell_start,
                                                             const uint32_t* __restrict__ sums,
                                                             uint32_t* __restrict__ dirty_list,
                                                             uint32_t* __restrict__ aoff, uint32_t ntiles) {
    __shared__ uint32_t s_data[kScanTile + kScanTile / 32];
    __shared__ uint32_t s_wave[3][kScanThreads / 64];
    __shared__ uint32_t s_pre[3][kScanThreads / 64];
    const uint32_t total = g->total_super;
    const uint32_t tile = blockIdx.x;
    const uint32_t needed = (total + kScanTile - 1) / kScanTile;
    const bool fused = needed <= kFusedScanTiles;
    if (fused && tile == 0 && threadIdx.x == 0 && needed > ntiles) raise_error(g, kErrInternal);
    if (tile * uint32_t(kScanTile) >= total || tile >= ntiles) return;
    const bool inc = g->inc != 0u;
    const int ncomp = inc ? 3 : 1;
    const uint32_t base = tile * kScanTile;
    const int wave = int(threadIdx.x >> 6);
    uint32_t pre[3] = {0u, 0u, 0u};
    if (fused) {   // the sums of the tiles before this one
        for (uint32_t t = threadIdx.x; t < tile; t += kScanThreads)
            for (int c = 0; c < ncomp; ++c) pre[c] += sums[c * ntiles + t];
        for (int c = 0; c < ncomp; ++c) {
            for (int d = 32; d >= 1; d >>= 1) pre[c] += __shfl_xor(pre[c], d, 64);
            if (lane_id() == 0) s_pre[c][wave] = pre[c];
        }
    }
    uint32_t v[kScanItems], dm;
    load_tile(in, g->epoch, inc, false, base, total, s_data, v, &dm);
    uint32_t x[3], run[3];
    thread_sums(v, dm, x);
    for (int c = 0; c < 3; ++c) {
        const uint32_t incl = wave_inclusive(x[c]);
        if (lane_id() == 63) s_wave[c][wave] = incl;
        run[c] = incl - x[c];
    }
    __syncthreads();
    for (int c = 0; c < ncomp; ++c) {
        if (fused) {
            for (int w = 0; w < kScanThreads / 64; ++w) run[c] += s_pre[c][w];
        } else {
            run[c] += sums[c * ntiles + tile];
        }
        for (int w = 0; w < wave; ++w) run[c] += s_wave[c][w];
    }
    const uint32_t g0 = base + threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; ++k) {
        s_data[lds_pad(threadIdx.x * kScanItems + k)] = run[0];
        if ((dm >> k) & 1u) {   // a changed super-box (update build only)
            dirty_list[run[1]] = g0 + k;
            aoff[g0 + k] = run[2];
            run[1] += 1u;
            run[2] += v[k];
        }
        run[0] += v[k];
    }
    // the last thread of the last tile ends with the totals
    if (fused && tile + 1 == needed && threadIdx.x == kScanThreads - 1) {
        cell_start[total] = run[0];
        if (inc) {
            g->ndirty = run[1];
            g->napp = run[2];
        }
    }
    __syncthreads();
    for (int k = 0; k < kScanItems / 4; ++k) {
        const uint32_t e4 = uint32_t(k) * kScanThreads + threadIdx.x;
        const uint32_t q0 = base + 4 * e4;
        uint32_t o[4];
        for (int c = 0; c < 4; ++c) o[c] = s_data[lds_pad(4 * e4 + c)];
        if (q0 + 4 <= total) {
            reinterpret_cast<uint4*>(cell_start)[q0 >> 2] = make_uint4(o[0], o[1], o[2], o[3]);
            reinterpret_cast<uint4*>(count)[q0 >> 2] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int c = 0; c < 4; ++c)
                if (q0 + c < total) {
                    cell_start[q0 + c] = o[c];
                    count[q0 + c] = 0u;
                }
        }
    }
}

// ------------------------------------------------------------------ scatter / fixup
// [st, en) is a slot range inside [0, n) (checked without wrap-around, so a
// corrupted start array cannot lead to accesses out of bounds).
__device__ __forceinline__ bool slot_range(uint32_t st, uint32_t en, uint32_t n) { return st <= en && en <= n; }

// The scatter writes, per agent of a (re)built super-box, a record {storage
// index, agent id, first canonical slot of the super-box, agent count << 4 |
// octant << 1 | moved} at a canonical slot of that super-box, so that the
// fixup finds everything it needs in the records of its super-box.  A full
// build rebuilds every super-box.  An update build rebuilds the changed ones
// (the list made by k_keys): their agents that stayed, found in their old
// storage ranges (which the update leaves dead), and the movers.
template <class T>
__global__ void k_scatter(Buffers<T> b, int cur, int ids_cur) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const uint32_t* __restrict__ cs = b.cell_start;
    if (!b.g->inc) {
        const uint32_t total = b.g->total_super;
        for (uint32_t i = tid; i < b.n; i += stride) {
            const SimGrid& G = b.sims[sim_index(b, i)];
            if (!G.valid) continue;
            const uint32_t key = b.key[i];
            const uint32_t sk = key >> 3;
            if (sk >= total) {
                raise_error(b.g, kErrInternal);
                continue;
            }
            const uint32_t st = cs[sk], en = cs[sk + 1], sub = b.sub[i];
            if (!slot_range(st, en, b.n) || sub >= en - st) {
                raise_error(b.g, kErrInternal);
                continue;
            }
            const uint32_t slot = st + sub;
            b.rec[slot] = make_uint4(i, b.ids[ids_cur][i], st,
                                     ((en - st) << 4) | ((key & 7u) << 1) | (b.flags[cur][i] & kMovedBit));
        }
        return;
    }
    // changed super-boxes, kFixupLanes threads each: the agents that stayed
    // (arrival counter: the super-box's count, which the scan left at zero)
    const uint32_t nd = b.g->ndirty;
    const uint32_t groups = stride / kFixupLanes, x0 = tid % kFixupLanes;
    for (uint32_t d = tid / kFixupLanes; d < nd; d += groups) {
        const uint32_t sk = b.dirty_list[d];
        const uint32_t o0 = b.cell_start_old[sk], o1 = b.cell_start_old[sk + 1];
        const uint32_t st = cs[sk], en = cs[sk + 1];
        if (!slot_range(o0, o1, b.n) || !slot_range(st, en, b.n)) {
            raise_error(b.g, kErrInternal);
            continue;
        }
        const uint32_t cnt = en - st;
        for (uint32_t u = o0 + x0; u < o1; u += kFixupLanes) {
            const uint32_t kold = b.skey[cur][u], fl = b.flags[cur][u];
            if (!(fl & kBoxChangedBit) || b.key[u] == kold) {
                const uint32_t r = atomicAdd(&b.count[sk], 1u);
                if (r < cnt)
                    b.rec[st + r] = make_uint4(u, b.ids[ids_cur][u], st,
                                               (cnt << 4) | ((kold & 7u) << 1) | (fl & kMovedBit));
                else
                    raise_error(b.g, kErrInternal);
            }
            b.skey[cur][u] = kDeadKey;   // the agent's loose slot is in the append region now
        }
    }
    // ... and the agents that entered another super-box, from the segments
    // of the keys kernel's blocks, one wave per segment
    const uint32_t kblocks = (b.n + kKeysSpan - 1) / kKeysSpan;
    const uint32_t waves = stride >> 6;
    for (uint32_t kb = tid >> 6; kb < kblocks; kb += waves) {
        const uint32_t mc = min(b.mcount[kb], kKeysSpan);
        for (uint32_t m0 = 0; m0 < mc; m0 += 64u) {   // wave-uniform: runs of equal super-boxes share an atomic
            const uint32_t m = m0 + uint32_t(lane_id());
            uint32_t i = 0, key = 0, sk = 0, st = 0, en = 0;
            bool act = false;
            if (m < mc) {
                i = b.movers[kb * kKeysSpan + m];
                if (i >= b.n) {
                    raise_error(b.g, kErrInternal);
                } else if (b.sub[i]) {
                    key = b.key[i];
                    sk = key >> 3;
                    if (sk >= b.g->total_super) {
                        raise_error(b.g, kErrInternal);
                    } else {
                        st = cs[sk];
                        en = cs[sk + 1];
                        act = slot_range(st, en, b.n);
                        if (!act) raise_error(b.g, kErrInternal);
                    }
                }
            }
            const uint32_t r = wave_run_add(b.count, act, sk);
            if (!act) continue;
            const uint32_t cnt = en - st;
            if (r >= cnt) {
                raise_error(b.g, kErrInternal);
                continue;
            }
            b.rec[st + r] =
                make_uint4(i, b.ids[ids_cur][i], st, (cnt << 4) | ((key & 7u) << 1) | (b.flags[cur][i] & kMovedBit));
        }
    }
}

// The simulation whose table range holds super-box sk: several simulations
// own fixed ranges in order of their sbase; one owns all.
__device__ __forceinline__ int sim_of_super(const SimGrid* sims, int nsims, uint32_t sk) {
    int lo = 0, hi = nsims - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sims[mid].sbase <= sk)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Rank of the agent of record slot t inside its super-box sk (records [st,
// st + cnt)) by (octant, id); the agent goes to loose slot x + rank, x the
// super-box's first loose slot.  When the step re-lays agents out (ids_next
// >= 0), its id and key also go to its canonical slot st + rank of the next
// state.  The first agent in that order writes the super-box's table entry.
template <class T>
__device__ __forceinline__ void fixup_slot(const Buffers<T>& b, const SimGrid& G, int cur, int ids_next, uint32_t t,
                                           uint32_t sk, uint32_t x) {
    const uint4 me = b.rec[t];
    const uint32_t i = me.x, st = me.z, cnt = me.w >> 4;
    if (i >= b.n || st > b.n || cnt > b.n - st || t < st || t - st >= cnt || x < b.n || x - b.n > b.n - cnt) {
        raise_error(b.g, kErrInternal);
        return;
    }
    // the agent's own state, requested before the walk over its super-box
    V4<T> p = pos4_ptr(b, cur)[i];
    const uint32_t fl = b.flags[cur][i];
    const unsigned long long mine = ((unsigned long long)((me.w >> 1) & 7u) << 32) | me.y;
    uint32_t r = 0, c2 = 0, c4 = 0, c6 = 0, moved = 0;
    // the super-box's records, four requested together
    for (uint32_t u0 = st; u0 < st + cnt; u0 += 4) {
        uint4 o4[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) o4[c] = b.rec[min(u0 + uint32_t(c), st + cnt - 1u)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint4& o = o4[c];
            const uint32_t in = u0 + uint32_t(c) < st + cnt ? 1u : 0u;
            const uint32_t oc = (o.w >> 1) & 7u;
            r += in & ((((unsigned long long)oc << 32) | o.y) < mine ? 1u : 0u);
            c2 += in & (oc < 2u ? 1u : 0u);
            c4 += in & (oc < 4u ? 1u : 0u);
            c6 += in & (oc < 6u ? 1u : 0u);
            moved |= (in & o.w) << oc;   // bit oc: an agent of octant oc moved
        }
    }
    const uint32_t u = x + r;
    const uint32_t key = (sk << 3) | ((me.w >> 1) & 7u);
    p.w = T(fabs(double(p.w)));
    if (fl & kMovedBit) p.w = -p.w;   // the walk reads the moved flag from the sign of d
    pos4_ptr(b, cur)[u] = p;
    b.flags[cur][u] = fl;
    b.skey[cur][u] = key;
    b.perm[u - b.n] = i;
    if (ids_next >= 0) {
        b.ids[ids_next][st + r] = me.y;
        b.skey[cur ^ 1][st + r] = key;
    }
    if (r == 0) {
        uint32_t q[3];
        if (!box_of<T>(G, p, q)) {
            raise_error(b.g, kErrInternal);
            return;
        }
        if (cnt > kMaxSuperCount) raise_error(b.g, kErrGrid);
        const uint32_t idx = super_index(G, q[0] >> 1, q[1] >> 1, q[2] >> 1);
        b.cellinfo[idx] = pack_super(x, cnt, c2, c4, c6, moved, G.stamp);
        b.tabidx[sk] = idx;
    }
}

// Full build: every canonical slot t, its agent to loose slot n + t (agents
// of a simulation whose grid overflowed keep their storage slot, state
// unchanged).  Update build: the changed super-boxes (the list made by the
// scan), kFixupLanes threads each, at their append slots.
template <class T>
__global__ void k_fixup(Buffers<T> b, int cur, int ids_next) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const uint32_t* __restrict__ cs = b.cell_start;
    if (!b.g->inc) {
        for (uint32_t t = tid; t < b.n; t += stride) {
            const SimGrid& G = b.sims[sim_index(b, t)];   // a simulation's slots are its agents' range
            if (G.valid) {
                const uint32_t i = b.rec[t].x;
                if (i >= b.n) {
                    raise_error(b.g, kErrInternal);
                    continue;
                }
                const uint32_t sk = b.key[i] >> 3;
                if (sk >= b.g->total_super) {
                    raise_error(b.g, kErrInternal);
                    continue;
                }
                fixup_slot<T>(b, G, cur, ids_next, t, sk, b.n + cs[sk]);
            } else {
                pos4_ptr(b, cur)[b.n + t] = pos4_ptr(b, cur)[t];
                b.flags[cur][b.n + t] = b.flags[cur][t];
                b.skey[cur][b.n + t] = kDeadKey;
                b.perm[t] = t;
                if (ids_next >= 0) {
                    b.ids[ids_next][t] = b.ids[ids_next ^ 1][t];
                    b.skey[cur ^ 1][t] = kDeadKey;
                }
            }
        }
        return;
    }
    // changed super-boxes, kFixupLanes threads each, at their append slots;
    // the super-box's count (the scatter's arrival counter) returns to zero
    const uint32_t nd = b.g->ndirty;
    const uint32_t groups = stride / kFixupLanes, x0 = tid % kFixupLanes;
    for (uint32_t d = tid / kFixupLanes; d < nd; d += groups) {
        const uint32_t sk = b.dirty_list[d];
        const uint32_t st = cs[sk], en = cs[sk + 1], cnt = en - st;
        const uint32_t a0 = b.aoff[sk];
        if (!slot_range(st, en, b.n) || a0 > b.n - cnt) {
            raise_error(b.g, kErrInternal);
            continue;
        }
        if (x0 == 0) b.count[sk] = 0u;
        if (cnt == 0) {   // emptied (so not empty in the last grid, which wrote its table index)
            if (x0 == 0) {
                // a rebuilt simulation's old entries are stale by its new
                // stamp, and their indices may be new super-boxes' now
                const SimGrid& G = b.sims[sim_of_super(b.sims, b.nsims, sk)];
                const uint32_t idx = b.tabidx[sk];
                if (idx >= b.g->total_super)
                    raise_error(b.g, kErrInternal);
                else if (!G.rebuild)
                    b.cellinfo[idx] = pack_super(0u, 0u, 0u, 0u, 0u, 0u, G.stamp);
            }
            continue;
        }
        for (uint32_t t = st + x0; t < st + cnt; t += kFixupLanes) {
            const SimGrid& G = b.sims[sim_index(b, t)];
            fixup_slot<T>(b, G, cur, ids_next, t, sk, b.n + a0);
        }
    }
}

__global__ void k_clear_u64(unsigned long long* p, uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_reset_stamp(Globals* g) { g->stamp = 0; }

template <class T>
void launch_clear_cellinfo(const Buffers<T>& b, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_stamp, dim3(1), dim3(1), 0, s, b.g);
    const uint64_t n = 2ull * b.super_capacity;   // 16-byte entries
    hipLaunchKernelGGL(k_clear_u64, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(b.cellinfo), n);
}

// ------------------------------------------------------------------ rank queries
// The agent in loose slot u of the last grid, if any: its storage index.
template <class T>
__device__ __forceinline__ bool loose_agent(const Buffers<T>& b, uint32_t u, uint32_t* i) {
    if (u < b.n) {
        *i = u;
        return b.g->inc && b.gkey[u] != kDeadKey;
    }
    if (u - b.n >= min(b.g->napp, b.n)) return false;
    *i = b.perm[u - b.n];
    return true;
}

// Gap-free rank (plus the simulation's box base) of the box of every agent of
// the last grid, from the positions that grid was built from, by id.  In
// Hilbert order: the boxes of the super-boxes the curve visits first, plus
// the box's Morton rank among the in-space boxes of its own super-box.
template <class T>
__global__ void k_box_ranks(Buffers<T> b, int ids_cur, uint32_t* __restrict__ out) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t i = 0;
    if (u >= 2u * b.n || !loose_agent(b, u, &i)) return;
    const uint32_t id = i < b.n ? b.ids[ids_cur][i] : 0xFFFFFFFFu;
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const SimGrid& G = b.sims[sim_index(b, i)];
    uint32_t rank = 0xFFFFFFFFu;
    uint32_t q[3];
    if (G.valid && box_of<T>(G, gpos_ptr(b)[u], q)) {
        if (b.hil) {
            const uint32_t S[3] = {q[0] >> 1, q[1] >> 1, q[2] >> 1};
            rank = G.box_base +
                   hilbert_rank(S[0], S[1], S[2], G.dims[0], G.dims[1], G.dims[2], G.slevels, 2u, b.hil->before,
                                b.hil->next) +
                   gapfree_rank(q[0] & 1u, q[1] & 1u, q[2] & 1u, min(2u, G.dims[0] - 2u * S[0]),
                                min(2u, G.dims[1] - 2u * S[1]), min(2u, G.dims[2] - 2u * S[2]), 1);
        } else {
            rank = G.box_base + gapfree_rank(q[0], q[1], q[2], G.dims[0], G.dims[1], G.dims[2], G.levels);
        }
    }
    out[id] = rank;
}

template <class T>
void launch_box_ranks(const Buffers<T>& b, int ids_cur, uint32_t* out, hipStream_t s) {
    const uint32_t m = 2u * b.n;
    hipLaunchKernelGGL(k_box_ranks<T>, dim3((m + 255) / 256), dim3(256), 0, s, b, ids_cur, out);
}

// Canonical order of the last grid: out[slot] = id.  The slot of an agent is
// its super-box's start cs[sk] plus its offset in the super-box's loose range.
template <class T>
__global__ void k_canonical_ids(Buffers<T> b, int ids_cur, const uint32_t* __restrict__ cs, uint32_t* __restrict__ out) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t i = 0;
    if (u >= 2u * b.n || !loose_agent(b, u, &i)) return;
    const uint32_t id = i < b.n ? b.ids[ids_cur][i] : 0xFFFFFFFFu;
    const SimGrid& G = b.sims[sim_index(b, i < b.n ? i : 0u)];
    uint32_t q[3];
    if (id >= b.n || !G.valid || !box_of<T>(G, gpos_ptr(b)[u], q)) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t x = b.cellinfo[super_index(G, q[0] >> 1, q[1] >> 1, q[2] >> 1)].x;
    const uint32_t sk = b.gkey[u] >> 3;
    const uint32_t t = sk < b.g->total_super ? cs[sk] + (u - x) : b.n;
    if (u < x || t >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    out[t] = id;
}

template <class T>
void launch_canonical_ids(const Buffers<T>& b, int ids_cur, const uint32_t* cs, uint32_t* out, hipStream_t s) {
    const uint32_t m = 2u * b.n;
    hipLaunchKernelGGL(k_canonical_ids<T>, dim3((m + 255) / 256), dim3(256), 0, s, b, ids_cur, cs, out);
}

// Grid of the kernels that loop over agents or changed super-boxes.
constexpr uint32_t kLoopBlocks = 8192;

template <class T>
void launch_grid(const Buffers<T>& b, int pos_cur, int ids_cur, bool relayout, bool moved_bits, hipStream_t s,
                 hipEvent_t* const* marks) {
    const uint32_t blocks = (b.n + 255) / 256;
    const uint32_t loop_blocks = blocks < kLoopBlocks ? blocks : kLoopBlocks;
    auto mark = [&](int k) {
        if (marks) (void)hipEventRecord(*marks[k], s);
    };
    hipLaunchKernelGGL(k_keys<T>, dim3((b.n + kKeysSpan - 1) / kKeysSpan), dim3(kKeysThreads), 0, s, b,
                       pos_cur, moved_bits ? 1 : 0);
    mark(0);
    const ScanIn in{b.count, b.cell_start_old, b.dirty, b.tabidx, b.mmask, b.cellinfo};
    hipLaunchKernelGGL(k_scan_reduce, dim3(b.scan_tiles), dim3(kScanThreads), 0, s, b.g, in, b.tile_sums,
                       b.scan_tiles);
    if (b.scan_tiles > kFusedScanTiles)   // else the rescan adds up the tile sums itself
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kTileScanThreads), 0, s, b.g, b.tile_sums, b.cell_start,
                           b.scan_tiles);
    hipLaunchKernelGGL(k_scan_down, dim3(b.scan_tiles), dim3(kScanThreads), 0, s, b.g, in, b.count, b.cell_start,
                       b.tile_sums, b.dirty_list, b.aoff, b.scan_tiles);
    mark(1);
    hipLaunchKernelGGL(k_scatter<T>, dim3(loop_blocks), dim3(256), 0, s, b, pos_cur, ids_cur);
    mark(2);
    hipLaunchKernelGGL(k_fixup<T>, dim3(loop_blocks), dim3(256), 0, s, b, pos_cur, relayout ? ids_cur ^ 1 : -1);
    mark(3);
}

#define ABM_INSTANTIATE(T)                                                                                 \
    template void launch_pack<T>(const Buffers<T>&, const T*, const T*, hipStream_t);                    \
    template void launch_occupied_boxes<T>(const Buffers<T>&, const int32_t*, const uint32_t*, uint32_t*,      \
                                           uint64_t, unsigned long long*, hipStream_t);                          \
    template void launch_radius<T>(const Buffers<T>&, int, hipStream_t);                                 \
    template void launch_finish_radius<T>(const Buffers<T>&, hipStream_t);                               \
    template void launch_extent<T>(const T*, const T*, uint32_t, Globals*, SimGrid*, hipStream_t);       \
    template void launch_mark_moved<T>(const Buffers<T>&, int, hipStream_t);                             \
    template void launch_bbox<T>(const Buffers<T>&, int, int, hipStream_t);                              \
    template void launch_reset_bbox<T>(const Buffers<T>&, int, hipStream_t);                             \
    template void launch_setup<T>(const Buffers<T>&, int, bool, hipStream_t);                            \
    template void launch_grid<T>(const Buffers<T>&, int, int, bool, bool, hipStream_t, hipEvent_t* const*); \
    template void launch_clear_cellinfo<T>(const Buffers<T>&, hipStream_t);                              \
    template void launch_box_ranks<T>(const Buffers<T>&, int, uint32_t*, hipStream_t);                   \
    template void launch_canonical_ids<T>(const Buffers<T>&, int, const uint32_t*, uint32_t*, hipStream_t);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
