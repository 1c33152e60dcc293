// abm_device.h -- device helpers shared by the libabm kernels.
#pragma once

#include "abm_internal.h"

namespace abm {

template <class T> struct Vec4Of;
template <> struct Vec4Of<float> { using type = float4; };
template <> struct Vec4Of<double> { using type = double4; };
template <class T> using V4 = typename Vec4Of<T>::type;

template <class T>
__device__ __forceinline__ V4<T>* pos4_ptr(const Buffers<T>& b, int which) {
    return reinterpret_cast<V4<T>*>(b.pos4[which]);
}

template <class T>
__device__ __forceinline__ int sim_index(const Buffers<T>& b, uint32_t i) {
    return b.sim_of ? int(b.sim_of[i]) : 0;
}

// Box coordinate floor(x / edge) along one axis, evaluated in double from the
// stored value (Section 3.1: the box of an agent follows from its position in
// constant time).  Returns false when the coordinate leaves the int32 range.
__device__ __forceinline__ bool box_coord(double x, double inv_h, int32_t* c) {
    const double v = floor(x * inv_h);
    if (!(v >= -2147483648.0 && v < 2147483647.0)) return false;
    *c = int32_t(v);
    return true;
}

// Gap-free Morton rank of box q inside a dims box (x in the lowest bit of the
// interleave).  Computed as the number of boxes of the space that precede q in
// Morton order: walking from the root of the implicit octree down to q, add
// the in-space boxes of every sibling subtree that comes before q's child.
// With r the in-space width of the current node from its origin (per axis),
// the node spans min(r, 2h) and its lower half min(r, h) boxes, h = 2^level,
// so a subtree's in-space boxes are a product of three such widths and no
// table is needed.  Requires dims[0]*dims[1]*dims[2] < 2^32 and
// 2^levels >= max(dims).
__device__ __forceinline__ uint32_t gapfree_rank(uint32_t qx, uint32_t qy, uint32_t qz, uint32_t dx, uint32_t dy,
                                                 uint32_t dz, int levels) {
    uint32_t r = 0, rx = dx, ry = dy, rz = dz;
    for (int lev = levels - 1; lev >= 0; --lev) {
        const uint32_t h = 1u << lev;
        const uint32_t bx = (qx >> lev) & 1u, by = (qy >> lev) & 1u, bz = (qz >> lev) & 1u;
        const uint32_t Wx = min(rx, 2u * h), Wy = min(ry, 2u * h), Wz = min(rz, 2u * h);
        const uint32_t lx = min(rx, h), ly = min(ry, h), lz = min(rz, h);
        const uint32_t wy = by ? Wy - ly : ly, wz = bz ? Wz - lz : lz;
        if (bz) r += Wx * Wy * lz;   // the lower z half of the node
        if (by) r += Wx * ly * wz;   // the lower y half of q's z half
        if (bx) r += lx * wy * wz;   // the lower x half of q's y quarter
        rx -= bx ? h : 0u;
        ry -= by ? h : 0u;
        rz -= bz ? h : 0u;
    }
    return r;
}

__device__ __forceinline__ void raise_error(Globals* g, uint32_t bits) { atomicOr(&g->err, bits); }

// Blocks are handed to the 8 XCDs round-robin.  Remap them so that each XCD
// works on runs of `run` consecutive logical blocks (neighbouring slots share
// that XCD's L2), the runs dealt to the XCDs in turn, so that every XCD gets
// a share of every region of the slot range (the cost per slot varies with
// the region).  `launched` is a multiple of 8 * run.
__device__ __forceinline__ uint32_t xcd_block(uint32_t run) {
    const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;   // XCD, and its k-th block
    return ((k / run) * 8u + x) * run + k % run;
}
// Run length for a launch of `blocks` blocks (at most 64, at least one run
// per XCD).
inline uint32_t xcd_run(uint32_t blocks) {
    uint32_t run = blocks / 64u;
    return run < 1u ? 1u : (run > 64u ? 64u : run);
}
inline uint32_t xcd_grid(uint32_t blocks, uint32_t run) { return (blocks + 8u * run - 1u) / (8u * run) * (8u * run); }

__device__ __forceinline__ int lane_id() { return int(threadIdx.x & 63u); }

__device__ __forceinline__ int32_t wave_min(int32_t v) {
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ int32_t wave_max(int32_t v) {
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ void bbox_atomic(int32_t* t, const int32_t lo[3], const int32_t hi[3]) {
    for (int a = 0; a < 3; ++a) {
        atomicMin(&t[a], lo[a]);
        atomicMax(&t[3 + a], hi[a]);
    }
}

// Fold the box ranges [clo, chi] of the active threads of a block into the
// accumulator target(sim) (6 ints: min x,y,z then max x,y,z).  Waves reduce
// in registers, the block combines its waves in LDS, and one set of atomics
// per simulation present in the block goes out, so that same-address
// atomics stay few.  Every thread of the block must call this once.
template <class Target>
__device__ void bbox_fold_block(int sim, bool active, const int32_t clo[3], const int32_t chi[3], Target target) {
    __shared__ int32_t s_box[16][6];
    __shared__ int s_sim[16];
    const int wave = int(threadIdx.x >> 6);
    const int nwaves = int((blockDim.x + 63u) >> 6);
    const unsigned long long act = __ballot(active);
    int s0 = -1;
    bool uniform = false;
    if (act) {
        const int leader = __ffsll((long long)act) - 1;
        s0 = __shfl(sim, leader, 64);
        uniform = __ballot(active && sim != s0) == 0;
    }
    if (act && uniform) {
        int32_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = wave_min(active ? clo[a] : INT32_MAX);
            hi[a] = wave_max(active ? chi[a] : INT32_MIN);
        }
        if (lane_id() == 0) {
            s_sim[wave] = s0;
            for (int a = 0; a < 3; ++a) {
                s_box[wave][a] = lo[a];
                s_box[wave][3 + a] = hi[a];
            }
        }
    } else {
        if (active) bbox_atomic(target(sim), clo, chi);
        if (lane_id() == 0) s_sim[wave] = -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int cur = -1;
        int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int w = 0; w < nwaves; ++w) {
            const int s = s_sim[w];
            if (s < 0) continue;
            if (s != cur) {
                if (cur >= 0) bbox_atomic(target(cur), lo, hi);
                cur = s;
                for (int a = 0; a < 3; ++a) {
                    lo[a] = s_box[w][a];
                    hi[a] = s_box[w][3 + a];
                }
            } else {
                for (int a = 0; a < 3; ++a) {
                    lo[a] = min(lo[a], s_box[w][a]);
                    hi[a] = max(hi[a], s_box[w][3 + a]);
                }
            }
        }
        if (cur >= 0) bbox_atomic(target(cur), lo, hi);
    }
}

template <class Target>
__device__ void bbox_fold_block(int sim, bool active, const int32_t c[3], Target target) {
    bbox_fold_block(sim, active, c, c, target);
}

// Replica of the bbox accumulator that this block folds into.
template <class T>
__device__ __forceinline__ int32_t* bbox_replica(const Buffers<T>& b, int slot, int sim) {
    const uint32_t r = blockIdx.x % kReplicas;
    return b.bbox_rep + ((size_t(slot) * kReplicas + r) * size_t(b.nsims) + size_t(sim)) * 6;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Largest value per simulation, folded like bbox_fold_block.
template <class Target>
__device__ void max_fold_block(int sim, bool active, unsigned long long v, Target target) {
    __shared__ unsigned long long s_val[16];
    __shared__ int s_sim[16];
    const int wave = int(threadIdx.x >> 6);
    const int nwaves = int((blockDim.x + 63u) >> 6);
    const unsigned long long act = __ballot(active);
    int s0 = -1;
    bool uniform = false;
    if (act) {
        const int leader = __ffsll((long long)act) - 1;
        s0 = __shfl(sim, leader, 64);
        uniform = __ballot(active && sim != s0) == 0;
    }
    if (act && uniform) {
        const unsigned long long m = wave_max_u64(active ? v : 0ull);
        if (lane_id() == 0) {
            s_sim[wave] = s0;
            s_val[wave] = m;
        }
    } else {
        if (active) atomicMax(target(sim), v);
        if (lane_id() == 0) s_sim[wave] = -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int cur = -1;
        unsigned long long m = 0;
        for (int w = 0; w < nwaves; ++w) {
            const int s = s_sim[w];
            if (s < 0) continue;
            if (s != cur) {
                if (cur >= 0) atomicMax(target(cur), m);
                cur = s;
                m = s_val[w];
            } else {
                m = s_val[w] > m ? s_val[w] : m;
            }
        }
        if (cur >= 0) atomicMax(target(cur), m);
    }
}

}  // namespace abm
