// abm_internal.h -- device data structures and kernel launchers of libabm.
//
// Boxes of edge h = cell_factor * R are grouped into super-boxes, the aligned
// 2x2x2 blocks S = q >> 1.  The 8 boxes of a super-box are 8 consecutive
// Morton codes, so in the canonical (box rank, id) order a super-box's agents
// are one contiguous slot range, sorted by octant (x bit lowest) and then id.
// The grid build therefore counts and scans super-boxes, not boxes.
//
// The grid holds the agents in "loose" slots u in [0, 2n): the walk reads a
// super-box's agents at [x, x + count) of the loose position array, x taken
// from its table entry.  A full build writes every agent to n + its canonical
// slot.  An update build (after a step that re-laid the agents out, with the
// same box extent) leaves the agents of every super-box that neither gained
// nor lost agents where the last step wrote them, at storage slots [0, n),
// and writes the agents of the other super-boxes, in canonical order per
// super-box, to an append region [n, n + napp).  Storage slots of those
// super-boxes are marked dead (kDeadKey).
//
// Layout in HBM (one workspace, carved by abm_api.hip):
//   per agent, two copies (ping-pong between steps), over the loose slots:
//     pos4   {x, y, z, d} in the element type T (16 B for float, 32 B for
//            double); the sign of d is the moved flag of the agent (written
//            so by the step; a full build sets it from the flags)
//     flags  bit 0 moved, bit 1 static (last step), bit 2 left its box, bits 8.. non-zero pair terms
//     skey   key of the grid the slot's agent was ranked in: (global
//            super-box rank << 3) | octant
//   per agent, two copies over the storage slots [0, n):
//     ids    persistent agent id held by each storage slot
//     force  3 doubles (only with keep_forces)
//   per agent, one copy (rebuilt every step):
//     key    new key of an agent (full build: all; update: agents that left their box)
//     sub    arrival index of the agent in its super-box (histogram atomics)
//     rec    agents of the rebuilt super-boxes in arrival order per super-box, at
//            canonical slots: {storage index, id, super-box start, count << 4 | octant << 1 | moved}
//     (key, sub and rec, 24 B per agent, live only inside a grid build: the
//     host calls between steps (queries, state import, population changes)
//     use the same bytes as their staging area)
//     perm   storage index of loose slot n + j
//     movers storage slots of the agents that left their box (update
//            build), listed per block of 256 agents, + a count per block
//   per super-box (capacity = sum of the per-simulation box capacities):
//     count       histogram (or count changes); every scan leaves it zeroed
//     cell_start  exclusive prefix sum of the counts (+1 entry), two copies
//                 (this grid and the last)
//     dirty, dirty_list, aoff   bookkeeping of the update build
//     tabidx      table index of the super-box (written with its entry)
//     mmask       moved octants of a kept super-box, gathered by the keys
//                 kernel and moved into its table entry by the scan
//     cellinfo    row-major super-box table, 16 B per entry (SuperEntry); an
//                 entry whose stamp is not its simulation's current one is
//                 empty, so the table is never cleared between steps (the
//                 timestamp trick of Section 3.1; update builds keep the
//                 stamps, a simulation rebuilt inside one takes a fresh one)
//   per scan tile: three 32-bit sums.
//   the Hilbert order's tables (HilbertTables, 768 B).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hilbert_order.h"

namespace abm {

constexpr uint32_t kMovedBit = 1u;
constexpr uint32_t kStaticBit = 2u;
constexpr uint32_t kBoxChangedBit = 4u;   // the last step took the agent out of the box it was ranked in
constexpr int kNnzShift = 8;
constexpr uint32_t kDeadKey = 0xFFFFFFFFu;   // storage slot whose agent the update build moved to the append region
constexpr uint32_t kMaxBoxesPerAxis = 1u << 21;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
// Reductions over all agents (box extent, step statistics) fold into this
// many copies of their accumulator, chosen by block index, so that
// same-address atomics stay few; the per-step setup kernel combines them.
constexpr int kReplicas = 64;

// Device error bits (latched, cleared by abm_sync).
enum : uint32_t {
    kErrNonfinite = 1u,     // a position or diameter is not finite
    kErrGrid = 2u,          // grid larger than its capacity or 2^21 boxes per axis
    kErrInternal = 8u,      // an index left its range (should never fire)
    kErrRange = 16u,        // a caller's value out of range (added diameter above R, bad or repeated id)
};

struct SimGrid {
    // set at init / set_params
    double radius;          // interaction radius R
    double inv_h;           // 1 / (cell_factor * R)
    double r2;              // R * R
    double k, gamma, mu, f_adh, delta_max;
    double cell_factor;
    uint32_t agent_begin, agent_end;
    uint32_t cap;           // box capacity of this simulation
    uint32_t scap;          // super-box capacity of this simulation (its table range, several simulations)
    // set by the per-step setup kernel
    int32_t cmin[3];
    uint32_t dims[3];
    uint32_t nboxes;
    uint32_t box_base;      // first global box index of this simulation (rank queries)
    int32_t levels;         // smallest L with 2^L >= max(dims)
    uint32_t valid;
    uint32_t sdims[3];      // super-boxes per axis: (dims + 1) >> 1
    uint32_t nsuper;        // sdims[0] * sdims[1] * sdims[2]
    uint32_t sbase;         // first global super-box index of this simulation (several simulations: fixed
                            // at init, the sum of the capacities before it, so a simulation's table range
                            // does not move when another one's grid changes)
    int32_t slevels;        // smallest L with 2^L >= max(sdims)
    uint32_t stamp;         // stamp of this simulation's current table entries
    uint32_t rebuild;       // this step rebuilds this simulation's grid inside an update build of the others
    // min x,y,z then max x,y,z of the box coordinates (extent queries only;
    // the step keeps its accumulators in Buffers::bbox_rep)
    int32_t bbox[2][6];
    uint64_t radius_bits;   // max diameter as ordered bits (init only)
};

struct Globals {
    uint32_t err;
    uint32_t total_super;    // super-boxes of all simulations in this step's grid
    uint32_t stamp;          // the latest stamp given to table entries (1..32767; each simulation keeps its own)
    uint32_t inc;            // this step's grid is an update of the last one (see launch_grid)
    uint32_t epoch;          // counts grid builds (marks this step's changed super-boxes; never 0)
    uint32_t ndirty;         // changed super-boxes of an update build (dirty_list, from the scan)
    uint32_t napp;           // agents in the append region (an update: of the changed super-boxes; full: n)
    uint32_t rebuilt;        // simulations rebuilt inside this step's update build (several simulations)
    // per step parity and replica: agents skipped as static, agents moved
    unsigned long long stats[2][kReplicas][2];
    // ... the sum of the forces the step evaluated (Newton's third law makes
    // it zero up to rounding when every force is evaluated) and the largest
    // displacement (as ordered bits of a non-negative double)
    double fsum[2][kReplicas][3];
    unsigned long long dmax[2][kReplicas];
};

// One block's share of the step's reductions: the box extent of its agents'
// new positions (min x, y, z, max x, y, z) and its static and moved counts.
struct BlockPart {
    int32_t box[6];
    uint32_t n_static, n_moved;
    double fsum[3];               // sum of the forces the block evaluated
    unsigned long long dmax;      // largest displacement, ordered bits
};

// Pointers into the workspace, passed by value to kernels.
template <class T>
struct Buffers {
    Globals* g;
    SimGrid* sims;
    const uint16_t* sim_of;   // null for a single simulation
    int32_t nsims;
    uint32_t n;
    uint32_t super_capacity;  // super-boxes the per-super-box arrays hold (a bound from the box capacities)
    uint32_t scan_tiles;
    // per loose slot [0, 2n) (+ kSposPad positions)
    void* pos4[2];
    uint32_t* flags[2];
    uint32_t* skey[2];
    // per storage slot
    uint32_t* ids[2];
    double* force[2];         // null without keep_forces
    uint32_t* key;
    uint32_t* sub;
    uint4* rec;               // per canonical slot of a rebuilt super-box: {storage index, id, super-box start, count << 4 | octant << 1 | moved}
    uint32_t* perm;           // storage index of loose slot n + j
    uint32_t* movers;         // agents that left their box (update build): block b of the keys kernel lists its own at [256 b, ...)
    uint32_t* mcount;         // ... and their number, per block of the keys kernel
    // loose slots of the last grid (set by the host with the grid build):
    // positions and keys of the grid's pos4/skey copy
    void* gpos;
    const uint32_t* gkey;
    // per super-box
    uint32_t* count;          // histogram (full build) or change of the counts (update)
    uint32_t* cell_start;     // first slot of every super-box, this grid
    uint32_t* cell_start_old; // ... of the last grid
    uint32_t* dirty;          // epoch of the last build in which the super-box gained or lost agents
    uint32_t* dirty_list;     // the changed super-boxes of this build, in rank order
    uint32_t* aoff;           // first append slot (minus n) of a changed super-box
    uint32_t* tabidx;         // table index of the super-box, written with its entry
    uint32_t* mmask;          // octants that hold an agent that moved (update build; zero between builds)
    uint4* cellinfo;
    const HilbertTables* hil; // the Hilbert order's tables; null: Morton order
    uint32_t* tile_sums;      // per scan tile: agents, changed super-boxes, agents of changed super-boxes
    double* partials;         // per-block partial sums (adjoint)
    uint32_t partial_cap;
    // box extent accumulators [2 slots][kReplicas][nsims][6]: one slot is
    // read by a step's setup, the other filled by its move kernel
    int32_t* bbox_rep;
    // single simulation: the step kernel's per-block results (box extent of
    // the new positions, static and moved counts), one record per launched
    // block, folded into the replicas by a second kernel without atomics
    BlockPart* bpart;
    uint32_t bpart_cap;
};

// The contact tape of one step (a full build): per canonical slot t, the
// agent's position (as the grid holds it), its id and its contacts'
// canonical slots in the order the force sums them (row r of slot t at
// list[r * n + t], at most kTapeWidth rows); *worst gets the largest
// contact count of the step (a tape with worst > kTapeWidth is incomplete
// and not used).  Ids, not storage indices: a re-layout moves agents
// between storage slots from one step to the next.
constexpr uint32_t kTapeWidth = 32;
struct TapeStep {
    void* pos;          // V4<T>[n]
    uint32_t* ids;      // [n]
    uint32_t* cnt;      // [n]
    uint32_t* list;     // [kTapeWidth][n]
    uint32_t* worst;    // one word, cleared before the step
};

// Host-side description of which kernels to run for one step.
struct StepArgs {
    int parity;             // which bbox accumulator describes the current positions
    int pos_cur;            // which pos4/flags/skey/force buffer holds the state
    int ids_cur;            // which ids buffer holds the state
    bool relayout;          // write the new state in canonical slot order
    bool detect_static;
    bool keep_forces;
    bool full_only;         // the grid is a full build (no agent in storage slots)
    int block_size;
    int walk_chunk;         // 2 or 4 candidate slots tested together by the neighbour walk
    bool share;             // the 2-wide walk of one simulation shares out the wave's pair terms
    const uint32_t* cs;     // this grid's super-box starts
    TapeStep tape;          // the step's contacts are taped here (pos null: not taped)
};

constexpr uint32_t kStampPeriod = 32767;   // 15-bit stamps in the super-box table
// Entries past the end of the slot-ordered position array (read, never used,
// by the neighbour walk).
constexpr int kSposPad = 4;
// Super-box keys carry the octant in their low 3 bits.
constexpr uint32_t kMaxSuperBoxes = 1u << 29;

// ---- launchers (grid_kernels.hip)
template <class T> void launch_pack(const Buffers<T>& b, const T* pos, const T* diam, hipStream_t s);
// Occupied boxes of one simulation's initial grid into *out (bits: a zeroed
// bitmap of nwords 32-bit words, one bit per box of the dims box at lo).
template <class T> void launch_occupied_boxes(const Buffers<T>& b, const int32_t lo[3], const uint32_t dims[3],
                                              uint32_t* bits, uint64_t nwords, unsigned long long* out,
                                              hipStream_t s);
template <class T> void launch_radius(const Buffers<T>& b, int pos_cur, hipStream_t s);
template <class T> void launch_finish_radius(const Buffers<T>& b, hipStream_t s);
template <class T> void launch_extent(const T* pos, const T* diam, uint32_t n, Globals* g, SimGrid* sim, hipStream_t s);
template <class T> void launch_mark_moved(const Buffers<T>& b, int pos_cur, hipStream_t s);
void launch_set_params(SimGrid* sims, int nsims, double k, double gamma, double mu, double f_adh, double delta_max,
                       hipStream_t s);
template <class T> void launch_bbox(const Buffers<T>& b, int pos_cur, int parity, hipStream_t s);
template <class T> void launch_setup(const Buffers<T>& b, int parity, bool allow_inc, hipStream_t s);
template <class T> void launch_grid(const Buffers<T>& b, int pos_cur, int ids_cur, bool relayout, bool moved_bits,
                                    hipStream_t s, hipEvent_t* const* marks = nullptr);
template <class T> void launch_clear_cellinfo(const Buffers<T>& b, hipStream_t s);
template <class T> void launch_box_ranks(const Buffers<T>& b, int ids_cur, uint32_t* out, hipStream_t s);
template <class T> void launch_canonical_ids(const Buffers<T>& b, int ids_cur, const uint32_t* cs, uint32_t* out,
                                             hipStream_t s);
template <class T> void launch_reset_bbox(const Buffers<T>& b, int parity, hipStream_t s);

// ---- launchers (force_kernels.hip)
template <class T> void launch_force(const Buffers<T>& b, const StepArgs& a, hipStream_t s);
// Per-block records the step kernel of n agents may write (its largest grid).
uint32_t force_part_capacity(uint32_t n);
// Fold nparts block records into the replicas of the box extent (slot
// parity ^ 1) and of the step statistics (parity), without atomics.
template <class T> void launch_fold_parts(const Buffers<T>& b, uint32_t nparts, int parity, hipStream_t s);

template <class T> void launch_neighbors(const Buffers<T>& b, int ids_cur, uint32_t* counts, uint32_t* rows,
                                         uint32_t K, uint32_t* worst, hipStream_t s);
template <class T> void launch_unpack_positions(const Buffers<T>& b, int pos_cur, int ids_cur, T* out, hipStream_t s);
template <class T> void launch_unpack_field(const Buffers<T>& b, int pos_cur, int ids_cur, int field, void* out,
                                            hipStream_t s);
template <class T> void launch_load_positions(const Buffers<T>& b, int pos_cur, int ids_cur, const T* in,
                                              hipStream_t s);
template <class T> void launch_set_flags(const Buffers<T>& b, int pos_cur, int ids_cur, const uint8_t* moved,
                                         const int32_t* nnz, hipStream_t s);

// ---- launchers (population_kernels.hip)
void launch_scan_u32(uint32_t* a, uint32_t n, uint32_t* tsum, hipStream_t s);
uint32_t gscan_tiles(uint32_t n);
template <class T> void launch_add(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t n0, uint32_t m, const T* pos,
                                   const T* diam, hipStream_t s);
// phase 0 marks the ids (rm = work[0, cap)); phase 1 renumbers and compacts
// into the other pos/flags/force and ids copies.  work: 4 cap + gscan_tiles(cap) words.
template <class T> void launch_remove(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t m, const int64_t* ids,
                                      uint32_t* work, uint32_t cap, hipStream_t s, int phase);
void launch_set_population(SimGrid* sims, uint32_t n, hipStream_t s);
// phase 0 marks the ids (mk = n words) and checks ids and diameters; phase 1
// writes the diameters that changed and marks their agents as moved.
template <class T> void launch_set_diameters(const Buffers<T>& b, int pos_cur, int ids_cur, uint32_t m,
                                             const int64_t* ids, const T* diam, uint32_t* mk, hipStream_t s, int phase);

// ---- launchers (adjoint_kernels.hip)
template <class T> void launch_adj_tape(const Buffers<T>& b, int ids_cur, const TapeStep& tp, hipStream_t s);
template <class T> void launch_adj_tape_w(const Buffers<T>& b, const TapeStep& tp, const double* lam, double* w,
                                          hipStream_t s);
template <class T> void launch_adj_tape_gather(const Buffers<T>& b, const TapeStep& tp, const double* lam,
                                               const double* w, double* lam_out, hipStream_t s);
template <class T> void launch_adj_w(const Buffers<T>& b, int ids_cur, const double* lam, double* w, hipStream_t s);
template <class T> void launch_adj_gather(const Buffers<T>& b, int ids_cur, const double* lam, const double* w,
                                          double* lam_out, hipStream_t s);
template <class T> void launch_adj_finish(const Buffers<T>& b, int nblocks, double* dparams, hipStream_t s);
int adj_blocks(uint32_t n);

}  // namespace abm
