// population_kernels.hip -- adding and removing agents between steps
// (Section 3.2), changing their diameters, and a device-wide exclusive scan
// of 32-bit counts that the removal uses.
//
// Agent ids are the agents' indices in the population, 0..n-1.  Addition
// appends: the new agents take ids n, n+1, ... and the storage slots after
// the last one.  Removal keeps the ids dense the way Section 3.2 keeps the
// agent vector dense: with new_size = n - m, the removed ids below new_size
// are holes, and the kept ids at or above new_size fill them, the k-th hole
// (ascending) taking the k-th such id (ascending).  The storage slots are
// compacted in order; their order does not matter, since the next grid is a
// full build that orders the agents by (box, id).
#include "force_loop.h"

namespace abm {

// ------------------------------------------------------------------ scan
constexpr int kGScanThreads = 256;
constexpr int kGScanItems = 16;
constexpr uint32_t kGScanTile = kGScanThreads * kGScanItems;

uint32_t gscan_tiles(uint32_t n) { return (n + kGScanTile - 1) / kGScanTile; }

__device__ __forceinline__ uint32_t gscan_wave_inclusive(uint32_t x) {
    const int lane = lane_id();
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__global__ __launch_bounds__(kGScanThreads) void k_gscan_reduce(const uint32_t* __restrict__ a, uint32_t n,
                                                                 uint32_t* __restrict__ tsum) {
    __shared__ uint32_t s_wave[kGScanThreads / 64];
    const uint32_t base = blockIdx.x * kGScanTile;
    uint32_t x = 0;
    for (int k = 0; k < kGScanItems; ++k) {
        const uint32_t i = base + uint32_t(k) * kGScanThreads + threadIdx.x;
        x += i < n ? a[i] : 0u;
    }
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if (lane_id() == 0) s_wave[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kGScanThreads / 64; ++w) t += s_wave[w];
        tsum[blockIdx.x] = t;
    }
}

// One block: exclusive scan of the tile sums in place.
constexpr int kGScanTileThreads = 1024;
__global__ __launch_bounds__(kGScanTileThreads) void k_gscan_tiles(uint32_t* __restrict__ tsum, uint32_t ntiles) {
    __shared__ uint32_t s_wave[kGScanTileThreads / 64];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < ntiles; base += kGScanTileThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < ntiles ? tsum[i] : 0u;
        const uint32_t incl = gscan_wave_inclusive(x);
        const int wave = int(threadIdx.x >> 6);
        if (lane_id() == 63) s_wave[wave] = incl;
        __syncthreads();
        uint32_t off = s_carry;
        for (int w = 0; w < wave; ++w) off += s_wave[w];
        if (i < ntiles) tsum[i] = off + incl - x;
        __syncthreads();
        if (threadIdx.x == kGScanTileThreads - 1) s_carry = off + incl;
        __syncthreads();
    }
}

// Each thread takes 16 consecutive values of the tile.
__global__ __launch_bounds__(kGScanThreads) void k_gscan_down(uint32_t* __restrict__ a, uint32_t n,
                                                               const uint32_t* __restrict__ tsum) {
    __shared__ uint32_t s_wave[kGScanThreads / 64];
    const uint32_t g0 = blockIdx.x * kGScanTile + threadIdx.x * kGScanItems;
    uint32_t v[kGScanItems], x = 0;
    for (int k = 0; k < kGScanItems; ++k) {
        v[k] = g0 + k < n ? a[g0 + k] : 0u;
        x += v[k];
    }
    const uint32_t incl = gscan_wave_inclusive(x);
    const int wave = int(threadIdx.x >> 6);
    if (lane_id() == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t run = tsum[blockIdx.x] + incl - x;
    for (int w = 0; w < wave; ++w) run += s_wave[w];
    for (int k = 0; k < kGScanItems; ++k) {
        if (g0 + k < n) a[g0 + k] = run;
        run += v[k];
    }
}

// a[0, n) <- its exclusive prefix sums; tsum holds gscan_tiles(n) words.
void launch_scan_u32(uint32_t* a, uint32_t n, uint32_t* tsum, hipStream_t s) {
    if (n == 0) return;
    const uint32_t t = gscan_tiles(n);
    hipLaunchKernelGGL(k_gscan_reduce, dim3(t), dim3(kGScanThreads), 0, s, a, n, tsum);
    hipLaunchKernelGGL(k_gscan_tiles, dim3(1), dim3(kGScanTileThreads), 0, s, tsum, t);
    hipLaunchKernelGGL(k_gscan_down, dim3(t), dim3(kGScanThreads), 0, s, a, n, tsum);
}

// ------------------------------------------------------------------ addition
// The m agents pos (m x 3) / diam (m) join at storage slots and ids n0 + j:
// moved (no history), no pair terms, no force.  A diameter above the
// interaction radius would let contacts escape the neighbour search.
template <class T>
__global__ void k_add(Buffers<T> b, int cur, int ids_cur, uint32_t n0, uint32_t m, const T* __restrict__ pos,
                      const T* __restrict__ diam) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint32_t i = n0 + j;
    V4<T> p;
    p.x = pos[3 * size_t(j)];
    p.y = pos[3 * size_t(j) + 1];
    p.z = pos[3 * size_t(j) + 2];
    p.w = diam[j];
    const double d = double(p.w);
    if (!(d > 0.0) || !isfinite(d) || !isfinite(double(p.x)) || !isfinite(double(p.y)) || !isfinite(double(p.z)))
        raise_error(b.g, kErrNonfinite);
    if (d > b.sims[0].radius) raise_error(b.g, kErrRange);
    pos4_ptr(b, cur)[i] = p;
    b.flags[cur][i] = kMovedBit;
    b.ids[ids_cur][i] = i;
    if (b.force[cur])
        for (int c = 0; c < 3; ++c) b.force[cur][3 * size_t(i) + c] = 0.0;
}

template <class T>
void launch_add(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t n0, uint32_t m, const T* pos, const T* diam,
                hipStream_t s) {
    hipLaunchKernelGGL(k_add<T>, dim3((m + 255) / 256), dim3(256), 0, s, b, pos_cur, ids_cur, n0, m, pos, diam);
}

// ------------------------------------------------------------------ removal
__global__ void k_fill_u32(uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// rm[id] = 1 for the m ids; an id out of range or given twice is an error.
__global__ void k_mark_removed(const int64_t* __restrict__ ids, uint32_t m, uint32_t n, uint32_t* __restrict__ rm,
                               Globals* g) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int64_t id = ids[j];
    if (id < 0 || id >= int64_t(n)) {
        raise_error(g, kErrRange);
        return;
    }
    if (atomicExch(&rm[id], 1u) != 0u) raise_error(g, kErrRange);
}

// pf[id] = 1 for a hole (removed, below new_size) and for a filler (kept, at
// or above new_size); their exclusive prefix sums rank both in ascending
// order, fillers after the holes.
__global__ void k_hole_flags(const uint32_t* __restrict__ rm, uint32_t n, uint32_t new_size,
                             uint32_t* __restrict__ pf) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pf[i] = i < new_size ? rm[i] : 1u - rm[i];
}

__global__ void k_list_holes(const uint32_t* __restrict__ rm, const uint32_t* __restrict__ pf, uint32_t new_size,
                             uint32_t* __restrict__ holes) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < new_size && rm[i]) holes[pf[i]] = i;
}

// kp[s] = 1 for a storage slot whose agent stays.
template <class T>
__global__ void k_keep_flags(Buffers<T> b, int ids_cur, const uint32_t* __restrict__ rm, uint32_t* __restrict__ kp) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= b.n) return;
    const uint32_t id = b.ids[ids_cur][s];
    kp[s] = id < b.n ? 1u - rm[id] : 0u;
    if (id >= b.n) raise_error(b.g, kErrInternal);
}

// The kept agents go, in storage order, to slots kp[s] of the other copy of
// the state, under their new ids.
template <class T>
__global__ void k_compact(Buffers<T> b, int cur, int ids_cur, uint32_t new_size, const uint32_t* __restrict__ rm,
                          const uint32_t* __restrict__ pf, const uint32_t* __restrict__ holes,
                          const uint32_t* __restrict__ kp) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= b.n) return;
    const uint32_t id = b.ids[ids_cur][s];
    if (id >= b.n || rm[id]) return;
    const uint32_t nholes = pf[new_size];   // new_size < n: the holes precede it
    uint32_t nid = id;
    if (id >= new_size) {
        const uint32_t r = pf[id] - nholes;
        nid = r < nholes ? holes[r] : 0xFFFFFFFFu;
    }
    const uint32_t dst = kp[s];
    if (nid >= new_size || dst >= new_size) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const int nxt = cur ^ 1;
    pos4_ptr(b, nxt)[dst] = pos4_ptr(b, cur)[s];
    b.flags[nxt][dst] = b.flags[cur][s];
    b.ids[ids_cur ^ 1][dst] = nid;
    if (b.force[cur])
        for (int c = 0; c < 3; ++c) b.force[nxt][3 * size_t(dst) + c] = b.force[cur][3 * size_t(s) + c];
}

__global__ void k_set_population(SimGrid* sims, uint32_t n) { sims[0].agent_end = n; }

template <class T>
void launch_remove(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t m, const int64_t* ids, uint32_t* work,
                   uint32_t cap, hipStream_t s, int phase) {
    const uint32_t n = b.n, new_size = n - m;
    uint32_t* rm = work;
    uint32_t* pf = work + cap;
    uint32_t* holes = work + 2 * size_t(cap);
    uint32_t* kp = work + 3 * size_t(cap);
    uint32_t* tsum = work + 4 * size_t(cap);
    const dim3 g((n + 255) / 256), bl(256);
    if (phase == 0) {   // mark (the caller checks the ids before anything moves)
        hipLaunchKernelGGL(k_fill_u32, g, bl, 0, s, rm, n, 0u);
        hipLaunchKernelGGL(k_mark_removed, dim3((m + 255) / 256), bl, 0, s, ids, m, n, rm, b.g);
        return;
    }
    hipLaunchKernelGGL(k_hole_flags, g, bl, 0, s, rm, n, new_size, pf);
    launch_scan_u32(pf, n, tsum, s);
    hipLaunchKernelGGL(k_list_holes, g, bl, 0, s, rm, pf, new_size, holes);
    hipLaunchKernelGGL(k_keep_flags<T>, g, bl, 0, s, b, ids_cur, rm, kp);
    launch_scan_u32(kp, n, tsum, s);
    hipLaunchKernelGGL(k_compact<T>, g, bl, 0, s, b, pos_cur, ids_cur, new_size, rm, pf, holes, kp);
}

// ------------------------------------------------------------------ diameters
// New diameters between steps (growth, shrinking, the mother's half of a
// division).  The grid stays valid: boxes depend on positions only, and a
// diameter may not exceed the interaction radius, which is also the box edge.

// mk[id] = j + 1 for the j-th (id, diameter) pair; an id out of range or
// given twice is a range error, a diameter that is not finite and positive a
// non-finite one.
template <class T>
__global__ void k_mark_diameters(const int64_t* __restrict__ ids, const T* __restrict__ diam, uint32_t m, uint32_t n,
                                 uint32_t* __restrict__ mk, Globals* g) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double d = double(diam[j]);
    if (!(d > 0.0) || !isfinite(d)) raise_error(g, kErrNonfinite);
    const int64_t id = ids[j];
    if (id < 0 || id >= int64_t(n)) {
        raise_error(g, kErrRange);
        return;
    }
    if (atomicExch(&mk[id], j + 1u) != 0u) raise_error(g, kErrRange);
}

// One thread per storage slot; the agent there, if listed, takes its new
// diameter.  Without apply the diameter is only checked against the
// interaction radius of the agent's simulation.  With apply it is written,
// and an agent whose diameter changed counts as moved in the last step, in
// its flags and in the sign of its stored diameter: then neither it nor an
// agent within R of it is static in the next step (condition (ii) of
// Section 5; a smaller diameter can raise a pair force too, by deepening the
// attraction).
template <class T>
__global__ void k_set_diameters(Buffers<T> b, int cur, int ids_cur, const T* __restrict__ diam,
                                const uint32_t* __restrict__ mk, uint32_t m, int apply) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= b.n) return;
    const uint32_t id = b.ids[ids_cur][s];
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t j = mk[id];
    if (j == 0u) return;
    if (j > m) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const T d = diam[j - 1u];
    if (!apply) {
        if (double(d) > b.sims[sim_index(b, s)].radius) raise_error(b.g, kErrRange);
        return;
    }
    V4<T>* __restrict__ p = pos4_ptr(b, cur);
    if (d == T(fabs(double(p[s].w)))) return;
    p[s].w = -d;
    b.flags[cur][s] |= kMovedBit;
}

template <class T>
void launch_set_diameters(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t m, const int64_t* ids,
                          const T* diam, uint32_t* mk, hipStream_t s, int phase) {
    const uint32_t n = b.n;
    const dim3 g((n + 255) / 256), bl(256);
    if (phase == 0) {   // mark and check (the caller reads the errors before anything changes)
        hipLaunchKernelGGL(k_fill_u32, g, bl, 0, s, mk, n, 0u);
        hipLaunchKernelGGL(k_mark_diameters<T>, dim3((m + 255) / 256), bl, 0, s, ids, diam, m, n, mk, b.g);
        hipLaunchKernelGGL(k_set_diameters<T>, g, bl, 0, s, b, pos_cur, ids_cur, diam, mk, m, 0);
        return;
    }
    hipLaunchKernelGGL(k_set_diameters<T>, g, bl, 0, s, b, pos_cur, ids_cur, diam, mk, m, 1);
}

void launch_set_population(SimGrid* sims, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_population, dim3(1), dim3(1), 0, s, sims, n);
}

#define ABM_INSTANTIATE(T)                                                                                  \
    template void launch_add<T>(const Buffers<T>&, int, int, uint32_t, uint32_t, const T*, const T*,     \
                                hipStream_t);                                                            \
    template void launch_remove<T>(const Buffers<T>&, int, int, uint32_t, const int64_t*, uint32_t*,       \
                                   uint32_t, hipStream_t, int);                                         \
    template void launch_set_diameters<T>(const Buffers<T>&, int, int, uint32_t, const int64_t*, const T*, \
                                          uint32_t*, hipStream_t, int);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
