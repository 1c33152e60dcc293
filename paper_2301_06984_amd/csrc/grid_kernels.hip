// grid_kernels.hip -- uniform-grid build of one step (Section 3.1) with boxes
// in gap-free Morton order (Section 4.2, steps D-F):
//   bbox     box extent of the agents (per simulation)
//   setup    dims, box counts and box bases of every simulation
//   keys     box key of every agent + histogram (atomics)
//   scan     single-pass exclusive scan with decoupled look-back
//   scatter  agents into box order (arrival order inside a box)
//   fixup    canonical (box, id) order inside each box + row-major box table
#include "abm_device.h"

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

// Largest diameter per simulation, as the bits of a positive double (which
// order like unsigned integers).
template <class T>
__global__ void k_radius(Buffers<T> b, int cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const double d = double(pos4_ptr(b, cur)[i].w);
    if (d > 0.0 && isfinite(d))
        atomicMax(&b.sims[sim_index(b, i)].radius_bits, (unsigned long long)__double_as_longlong(d));
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

__global__ void k_reset_bbox(SimGrid* sims, int nsims, int slot);

// Extent of caller-layout positions (n x 3 + diameters) for sizing a grid:
// largest diameter, then box coordinates in the first bbox accumulator.
template <class T>
__global__ void k_extent_radius(const T* __restrict__ diam, uint32_t n, Globals* g, SimGrid* sim) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = double(diam[i]);
    if (!(d > 0.0) || !isfinite(d)) {
        raise_error(g, kErrNonfinite);
        return;
    }
    atomicMax(&sim->radius_bits, (unsigned long long)__double_as_longlong(d));
}

template <class T>
__global__ void k_extent_bbox(const T* __restrict__ pos, uint32_t n, Globals* g, SimGrid* sim) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = i < n;
    int32_t c[3] = {0, 0, 0};
    if (active) {
        const double ih = sim->inv_h;
        const bool ok = box_coord(double(pos[3 * size_t(i)]), ih, &c[0]) &&
                        box_coord(double(pos[3 * size_t(i) + 1]), ih, &c[1]) &&
                        box_coord(double(pos[3 * size_t(i) + 2]), ih, &c[2]);
        if (!ok) {
            raise_error(g, kErrNonfinite);
            active = false;
        }
    }
    bbox_accumulate(sim, 0, 0, active, c);
}

template <class T>
void launch_extent(const T* pos, const T* diam, uint32_t n, Globals* g, SimGrid* sim, hipStream_t s) {
    const uint32_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_extent_radius<T>, dim3(blocks), dim3(256), 0, s, diam, n, g, sim);
    hipLaunchKernelGGL(k_finish_radius, dim3(1), dim3(64), 0, s, sim, 1);
    hipLaunchKernelGGL(k_reset_bbox, dim3(1), dim3(64), 0, s, sim, 1, 0);
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

__global__ void k_reset_bbox(SimGrid* sims, int nsims, int slot) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsims) return;
    for (int a = 0; a < 3; ++a) {
        sims[s].bbox[slot][a] = INT32_MAX;
        sims[s].bbox[slot][3 + a] = INT32_MIN;
    }
}

template <class T>
void launch_reset_bbox(const Buffers<T>& b, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_bbox, dim3((b.nsims + 255) / 256), dim3(256), 0, s, b.sims, b.nsims, parity);
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
    bbox_accumulate(b.sims, sim, slot, active, c);
}

template <class T>
void launch_bbox(const Buffers<T>& b, int pos_cur, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_bbox, dim3((b.nsims + 255) / 256), dim3(256), 0, s, b.sims, b.nsims, parity);
    const uint32_t blocks = (b.n + 255) / 256;
    hipLaunchKernelGGL(k_bbox<T>, dim3(blocks), dim3(256), 0, s, b, pos_cur, parity);
}

// ------------------------------------------------------------------ setup
// One block: per simulation, dims and box count from its bbox accumulator,
// then an exclusive scan of the box counts gives each simulation's base in
// the shared box arrays.  Also clears the other accumulator for this step's
// move kernel and the step statistics.
constexpr int kSetupThreads = 1024;

__global__ __launch_bounds__(kSetupThreads) void k_setup(Globals* g, SimGrid* sims, int nsims, int parity,
                                                           uint32_t box_capacity) {
    __shared__ uint32_t s_wave[kSetupThreads / 64];
    __shared__ unsigned long long s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int chunk = 0; chunk < nsims; chunk += kSetupThreads) {
        const int s = chunk + int(threadIdx.x);
        uint32_t nb = 0;
        if (s < nsims) {
            SimGrid& G = sims[s];
            const int32_t* bb = G.bbox[parity];
            bool ok = true;
            uint64_t total = 1;
            int levels = 0;
            for (int a = 0; a < 3; ++a) {
                const int64_t lo = bb[a], hi = bb[3 + a];
                const int64_t d = hi - lo + 1;
                if (hi < lo || d > int64_t(kMaxBoxesPerAxis)) ok = false;
                const uint32_t du = ok ? uint32_t(d) : 1u;
                G.cmin[a] = int32_t(lo);
                G.dims[a] = du;
                total *= du;
                while ((1u << levels) < du) ++levels;
            }
            if (total > uint64_t(G.cap) || total >= (uint64_t(1) << 32)) ok = false;
            G.levels = levels;
            G.valid = ok ? 1u : 0u;
            G.nboxes = ok ? uint32_t(total) : 0u;
            nb = G.nboxes;
            if (!ok) raise_error(g, kErrGrid);
            for (int a = 0; a < 3; ++a) {
                G.bbox[parity ^ 1][a] = INT32_MAX;
                G.bbox[parity ^ 1][3 + a] = INT32_MIN;
            }
        }
        // block exclusive scan of nb
        uint32_t x = nb;
        const int lane = int(threadIdx.x & 63u), wave = int(threadIdx.x >> 6);
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) s_wave[wave] = x;
        __syncthreads();
        uint32_t wave_off = 0;
        for (int w = 0; w < wave; ++w) wave_off += s_wave[w];
        const unsigned long long base = s_carry + wave_off + x - nb;
        if (s < nsims) sims[s].box_base = uint32_t(base);
        __syncthreads();
        if (threadIdx.x == kSetupThreads - 1) s_carry = base + nb;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long total = s_carry;
        if (total > box_capacity) {
            raise_error(g, kErrGrid);
            total = 0;
            for (int s = 0; s < nsims; ++s) sims[s].valid = 0;
        }
        g->total_boxes = uint32_t(total);
        // a fresh stamp marks this step's box table entries (the host clears
        // the table before the 15-bit stamp wraps); a fresh epoch tags this
        // step's scan status words
        g->stamp = g->stamp + 1;
        g->scan_epoch = (g->scan_epoch % 0x3FFFFFFFu) + 1;
        g->n_static[parity] = 0;
        g->n_moved[parity] = 0;
    }
}

template <class T>
void launch_setup(const Buffers<T>& b, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(kSetupThreads), 0, s, b.g, b.sims, b.nsims, parity, b.box_capacity);
}

// ------------------------------------------------------------------ keys
template <class T>
__global__ void k_keys(Buffers<T> b, int cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const SimGrid& G = b.sims[sim_index(b, i)];
    if (!G.valid) return;
    const V4<T> p = pos4_ptr(b, cur)[i];
    int32_t c[3];
    const bool ok = box_coord(double(p.x), G.inv_h, &c[0]) && box_coord(double(p.y), G.inv_h, &c[1]) &&
                    box_coord(double(p.z), G.inv_h, &c[2]);
    uint32_t q[3];
    bool in = ok;
    for (int a = 0; a < 3; ++a) {
        const int64_t v = int64_t(c[a]) - int64_t(G.cmin[a]);
        in = in && v >= 0 && v < int64_t(G.dims[a]);
        q[a] = uint32_t(v);
    }
    if (!in) {  // the extent is computed from these very positions
        raise_error(b.g, kErrInternal);
        b.key[i] = 0xFFFFFFFFu;
        return;
    }
    const uint32_t rank = gapfree_rank(q[0], q[1], q[2], G.dims[0], G.dims[1], G.dims[2], G.levels);
    const uint32_t key = G.box_base + rank;
    b.key[i] = key;
    b.rmi[i] = G.box_base + (q[2] * G.dims[1] + q[1]) * G.dims[0] + q[0];
    b.sub[i] = atomicAdd(&b.count[key], 1u);
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

// Exclusive scan of count[0, total) into cell_start[0, total], zeroing count.
// Tiles take their position from a ticket, so a tile only waits on tiles that
// already run; each tile publishes its aggregate, then its inclusive prefix
// (status word: epoch | flag | value), and sums its predecessors' words.
__global__ __launch_bounds__(kScanThreads) void k_scan(Globals* g, uint32_t* __restrict__ count,
                                                        uint32_t* __restrict__ cell_start,
                                                        unsigned long long* status, uint32_t ntiles) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kScanThreads / 64];
    __shared__ uint32_t s_prefix;
    if (threadIdx.x == 0) s_tile = uint32_t(atomicAdd(&g->scan_ticket, 1ull) % ntiles);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t total = g->total_boxes;
    const uint32_t epoch = g->scan_epoch;
    const uint32_t needed = (total + kScanTile - 1) / kScanTile;
    if (needed > ntiles) {
        if (tile == 0 && threadIdx.x == 0) raise_error(g, kErrInternal);
        return;
    }
    if (tile >= needed) return;   // no tile waits on a later one
    const uint32_t first = tile * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    if (first + kScanItems <= total) {
        const uint4* src = reinterpret_cast<const uint4*>(count + first);
        for (int k = 0; k < kScanItems / 4; ++k) {
            const uint4 u = src[k];
            v[4 * k] = u.x; v[4 * k + 1] = u.y; v[4 * k + 2] = u.z; v[4 * k + 3] = u.w;
        }
    } else {
        for (int k = 0; k < kScanItems; ++k) v[k] = first + k < total ? count[first + k] : 0u;
    }
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    const uint32_t incl = wave_inclusive(sum);
    const int wave = int(threadIdx.x >> 6);
    if (lane_id() == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t wave_off = 0, agg = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wave) wave_off += s_wave[w];
        agg += s_wave[w];
    }
    if (threadIdx.x == 0) {
        const unsigned long long tag = (unsigned long long)(epoch & 0x3FFFFFFFu) << 34;
        uint32_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(&status[0], tag | (2ull << 32) | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[tile], tag | (1ull << 32) | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            int64_t p = int64_t(tile) - 1;
            uint32_t spins = 0;
            while (p >= 0) {
                const unsigned long long w =
                    __hip_atomic_load(&status[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t flag = uint32_t(w >> 32) & 3u;
                if (uint32_t(w >> 34) != (epoch & 0x3FFFFFFFu) || flag == 0) {
                    if (++spins > (1u << 26)) {   // a predecessor never published: give up loudly
                        raise_error(g, kErrInternal);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += uint32_t(w);
                if (flag == 2) break;
                --p;
            }
            __hip_atomic_store(&status[tile], tag | (2ull << 32) | (prefix + agg), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix = prefix;
        if (tile == needed - 1) cell_start[total] = prefix + agg;
    }
    __syncthreads();
    uint32_t run = s_prefix + wave_off + incl - sum;
    if (first + kScanItems <= total) {
        uint4* dst = reinterpret_cast<uint4*>(cell_start + first);
        uint4* zero = reinterpret_cast<uint4*>(count + first);
        for (int k = 0; k < kScanItems / 4; ++k) {
            uint4 o;
            o.x = run; run += v[4 * k];
            o.y = run; run += v[4 * k + 1];
            o.z = run; run += v[4 * k + 2];
            o.w = run; run += v[4 * k + 3];
            dst[k] = o;
            zero[k] = make_uint4(0u, 0u, 0u, 0u);
        }
    } else {
        for (int k = 0; k < kScanItems; ++k) {
            if (first + k < total) {
                cell_start[first + k] = run;
                count[first + k] = 0u;
            }
            run += v[k];
        }
    }
}

// ------------------------------------------------------------------ scatter / fixup
template <class T>
__global__ void k_scatter(Buffers<T> b) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    if (!b.sims[sim_index(b, i)].valid) return;
    const uint32_t key = b.key[i];
    if (key >= b.g->total_boxes) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t slot = b.cell_start[key] + b.sub[i];
    if (slot >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    b.tmp[slot] = i;
}

// Slot t holds agent tmp[t]; its final slot is the start of its box plus the
// number of agents of that box with a smaller id.  The first agent of each box
// writes the box's row-major table entry.
template <class T>
__global__ void k_fixup(Buffers<T> b, int cur, int ids_cur) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.n) return;
    if (!b.sims[sim_index(b, t)].valid) return;   // a simulation's slots are its agents' range
    const uint32_t i = b.tmp[t];
    if (i >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t c = b.key[i];
    if (c >= b.g->total_boxes) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t st = b.cell_start[c], en = b.cell_start[c + 1];
    if (en > b.n || st > en) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t* ids = b.ids[ids_cur];
    const uint32_t* fl = b.flags[cur];
    const uint32_t myid = ids[i];
    const uint32_t stamp = b.g->stamp;
    uint32_t r = 0, moved = 0;
    for (uint32_t u = st; u < en; ++u) {
        const uint32_t j = b.tmp[u];
        if (j >= b.n) continue;
        r += ids[j] < myid ? 1u : 0u;
        moved |= fl[j] & kMovedBit;
    }
    if (st + r >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    b.perm[st + r] = i;
    if (r == 0) {
        uint32_t cnt = en - st;
        if (cnt > 0xFFFFu) {
            raise_error(b.g, kErrBoxOverflow);
            cnt = 0xFFFFu;
        }
        b.cellinfo[b.rmi[i]] = pack_cell(st, cnt, stamp, moved);
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
    const uint64_t n = b.box_capacity;
    hipLaunchKernelGGL(k_clear_u64, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s, b.cellinfo, n);
    const uint64_t nt = b.scan_tiles;
    hipLaunchKernelGGL(k_clear_u64, dim3(uint32_t((nt + 255) / 256)), dim3(256), 0, s, b.scan_status, nt);
}

template <class T>
void launch_grid(const Buffers<T>& b, int pos_cur, int ids_cur, hipStream_t s) {
    const uint32_t blocks = (b.n + 255) / 256;
    hipLaunchKernelGGL(k_keys<T>, dim3(blocks), dim3(256), 0, s, b, pos_cur);
    hipLaunchKernelGGL(k_scan, dim3(b.scan_tiles), dim3(kScanThreads), 0, s, b.g, b.count, b.cell_start,
                       b.scan_status, b.scan_tiles);
    hipLaunchKernelGGL(k_scatter<T>, dim3(blocks), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_fixup<T>, dim3(blocks), dim3(256), 0, s, b, pos_cur, ids_cur);
}

#define ABM_INSTANTIATE(T)                                                                                 \
    template void launch_pack<T>(const Buffers<T>&, const T*, const T*, hipStream_t);                    \
    template void launch_radius<T>(const Buffers<T>&, int, hipStream_t);                                 \
    template void launch_finish_radius<T>(const Buffers<T>&, hipStream_t);                               \
    template void launch_extent<T>(const T*, const T*, uint32_t, Globals*, SimGrid*, hipStream_t);       \
    template void launch_mark_moved<T>(const Buffers<T>&, int, hipStream_t);                             \
    template void launch_bbox<T>(const Buffers<T>&, int, int, hipStream_t);                              \
    template void launch_reset_bbox<T>(const Buffers<T>&, int, hipStream_t);                             \
    template void launch_setup<T>(const Buffers<T>&, int, hipStream_t);                                  \
    template void launch_grid<T>(const Buffers<T>&, int, int, hipStream_t);                              \
    template void launch_clear_cellinfo<T>(const Buffers<T>&, hipStream_t);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
