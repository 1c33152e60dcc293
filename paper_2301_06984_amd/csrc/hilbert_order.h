// hilbert_order.h -- the Hilbert order of the super-boxes, the variant order
// next to Morton order (Section 4.2 compares the two space-filling curves).
//
// The aligned 2x2x2 blocks of boxes (super-boxes) follow a Hilbert curve over
// the smallest power-of-two cube that holds the super grid; the 8 boxes of a
// block keep Morton order (the force walk cuts a block's halves by octant
// counts, which needs that).  The curve is the one of Skilling's transform
// (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004),
// x its first coordinate.
//
// A rank is gap-free: the number of super-boxes inside the space that the
// curve visits first.  It is found by walking the implicit octree from the
// root to the super-box: at every node, add the in-space part of each child
// the curve visits before the one holding the super-box.  Which children
// those are depends only on the node's orientation, one of a few states; two
// small tables, built once on the host from the transform itself, give per
// (state, child) the children visited first (a bit mask) and the child's own
// state.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace abm {

constexpr int kHilMaxStates = 48;   // orientations of a cube, the most a curve can use

struct HilbertTables {
    uint8_t before[kHilMaxStates * 8];   // [state * 8 + child]: children visited first, bit c' for child c'
    uint8_t next[kHilMaxStates * 8];     // [state * 8 + child]: the child's state (the root is state 0)
};

// Fill t from the transform: false if the curve needs more states than the
// tables hold or a transition is not the same wherever it occurs (neither
// happens for a Hilbert curve; the check makes a wrong transform fail loudly).
bool build_hilbert_tables(HilbertTables* t);

__host__ __device__ inline uint32_t hil_min(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Gap-free Hilbert rank of the super-box (sx, sy, sz) whose space extends
// (ex, ey, ez) units from the origin, over 2^levels super-boxes per axis.
// unit = 1 counts super-boxes (extent = super-boxes per axis); unit = 2
// counts boxes (extent = boxes per axis), so that the rank is the number of
// boxes of the super-boxes visited first.  before and next are the tables'
// arrays (global memory or an LDS copy).
__host__ __device__ inline uint32_t hilbert_rank(uint32_t sx, uint32_t sy, uint32_t sz, uint32_t ex, uint32_t ey,
                                                 uint32_t ez, int levels, uint32_t unit, const uint8_t* before,
                                                 const uint8_t* next) {
    uint32_t r = 0, st = 0, rx = ex, ry = ey, rz = ez;
    for (int lev = levels - 1; lev >= 0; --lev) {
        const uint32_t h = unit << lev;   // a child's width in counted units
        const uint32_t bx = (sx >> lev) & 1u, by = (sy >> lev) & 1u, bz = (sz >> lev) & 1u;
        const uint32_t c = bx | (by << 1) | (bz << 2);
        // in-space widths of the lower and upper child along each axis
        const uint32_t lx = hil_min(rx, h), ly = hil_min(ry, h), lz = hil_min(rz, h);
        const uint32_t ux = hil_min(rx, 2u * h) - lx, uy = hil_min(ry, 2u * h) - ly, uz = hil_min(rz, 2u * h) - lz;
        const uint32_t m = before[st * 8u + c];
        for (uint32_t k = 0; k < 8u; ++k) {
            const uint32_t w = ((k & 1u) ? ux : lx) * ((k & 2u) ? uy : ly) * ((k & 4u) ? uz : lz);
            r += ((m >> k) & 1u) ? w : 0u;
        }
        st = next[st * 8u + c];
        rx -= bx ? h : 0u;
        ry -= by ? h : 0u;
        rz -= bz ? h : 0u;
    }
    return r;
}

}  // namespace abm
