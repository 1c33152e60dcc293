/*
 * abm.h -- C ABI of the MI355X agent-step library (libabm.so).
 *
 * One mechanical step of N spherical agents, the hot path of the agent-based
 * engine described in "High-Performance and Scalable Agent-Based Simulation
 * with BioDynaMo" (arXiv 2301.06984):
 *   - uniform grid with an O(1) box lookup from the position and a 3x3x3 box
 *     search (Section 3.1), boxes ranked in gap-free Morton order
 *     (Section 4.2, steps D-E) and agents sorted into array-based box lists;
 *   - the pairwise sphere-sphere collision force and the displacement it
 *     causes, with a force threshold (Section 5; force law: see below);
 *   - the skip of the force computation for static agents (Section 5);
 *   - agents re-laid out along the Morton curve every sort_every steps
 *     (Section 4.2, step G), or, as an option, with the 2x2x2 blocks of
 *     boxes along a Hilbert curve (the other curve Section 4.2 compares);
 *   - agents added, removed and given new diameters between steps
 *     (Section 3.2; conditions (ii) and (iii) of the static test, Section 5);
 *   - a batched form (many independent simulations per launch) and a
 *     reverse-mode (adjoint) form of the step.
 *
 * Force law (the paper defers to the Cortex3D method and does not print it):
 *   f(delta, rho) = k * delta - gamma * sqrt(rho * delta),
 *   delta = r_i + r_j - |x_i - x_j| > 0, rho = r_i r_j / (r_i + r_j),
 *   F_i = sum_j f * (x_i - x_j) / |x_i - x_j| over the neighbours j (|x_i - x_j| < R).
 * Displacement: if |F_i| > f_adh then Delta_i = mu F_i clamped to |Delta_i| <= delta_max,
 * else 0; all agents move after all forces are known (Jacobi update).
 *
 * Conventions for every function:
 *   - returns ABM_OK (0) or a negative ABM_E_* code; nothing throws across the ABI;
 *     abm_last_error() gives a message for the calling thread's last failure;
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory;
 *   - the caller owns every device buffer (inputs, workspace, outputs); the
 *     library never allocates device memory (graph objects aside) and keeps
 *     raw pointers into the workspace until abm_destroy(); its only device
 *     memory of its own is the fixed 1 KiB scratch of abm_extent_of_noalloc;
 *   - `stream` is a hipStream_t (0 = the null stream); all work is enqueued on
 *     it asynchronously; a context is bound to its stream and is not
 *     thread-safe;
 *   - positions are n x 3 row-major, diameters n; their element type is
 *     float (ABM_F32) or double (ABM_F64) as params.precision says;
 *     geometric tests and forces are evaluated in double in both modes, the
 *     stored state is rounded to the element type once per step.
 */
#ifndef ABM_H
#define ABM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABM_ABI_VERSION 6
#define ABM_EXTENT_SCRATCH_BYTES 1024

enum abm_status {
    ABM_OK = 0,
    ABM_E_INVAL = -1,        /* bad argument, size or alignment */
    ABM_E_NONFINITE = -2,    /* a non-finite input or state value */
    ABM_E_GRID = -3,         /* grid larger than 2^21 boxes per axis, 2^32 boxes, 2^29 super-boxes (aligned
                                2x2x2 blocks of boxes), or the box capacity */
    ABM_E_WORKSPACE = -4,    /* workspace too small */
    ABM_E_HIP = -5,          /* HIP runtime failure */
    ABM_E_STATE = -6,        /* call out of order (e.g. backward before a recorded forward) */
    ABM_E_UNSUPPORTED = -7   /* feature not available in this configuration */
};

enum abm_precision { ABM_F32 = 0, ABM_F64 = 1 };

/* Order of the boxes in memory (Section 4.2 compares the two space-filling curves). */
enum abm_order {
    ABM_ORDER_MORTON = 0,   /* gap-free Morton order of the boxes */
    ABM_ORDER_HILBERT = 1   /* the 2x2x2 blocks of boxes along a Hilbert curve (Skilling's transform, x first),
                               over the smallest power-of-two cube holding them; Morton order inside a block */
};

typedef struct abm_params {
    double k;                  /* repulsion coefficient (default 2) */
    double gamma;              /* adhesion coefficient (default 1) */
    double mu;                 /* mobility: displacement per unit force (default 0.1) */
    double f_adh;              /* force threshold that |F| must exceed to move (default 0) */
    double delta_max;          /* largest displacement per step (default 3) */
    double interaction_radius; /* R; 0 = the largest diameter (default 0) */
    double cell_factor;        /* box edge = cell_factor * R, >= 1 (default 1) */
    int32_t precision;         /* ABM_F32 or ABM_F64 */
    int32_t detect_static;     /* skip the force of static agents (Section 5) */
    int32_t sort_every;        /* re-lay out agents in Morton order every k steps; 0 = never */
    int32_t block_size;        /* threads per block of the force kernel: 64..1024, multiple of 64; 0 = 256 */
    int32_t keep_forces;       /* store F_i each step so ABM_FIELD_FORCES can be queried */
    int32_t walk_chunk;        /* candidates the neighbour walk tests together: 2 or 4; 0 = chosen at init
                                  from how densely the agents fill their boxes: one simulation, 4 at 4 or more
                                  agents per occupied box of the initial grid (clustered agents; no uniform
                                  packing reaches 3); a batch, 4 at 3 or more per box of the extent; else 2 */
    int32_t order;             /* ABM_ORDER_MORTON (default) or ABM_ORDER_HILBERT; fixed at init, the same for
                                  every simulation of a batch.  It sets the canonical order, and with it the
                                  order in which each agent's pair terms are summed */
    int32_t share_terms;       /* the 2-wide walk of one simulation: 1 = each lane adds its own agent's pair
                                  terms, 2 = the wave shares out all its lanes' pair terms, one per lane (the
                                  same sums, bit for bit; pays where agents have several contacts); 0 = chosen
                                  at init: 2 at 2 or more agents per occupied box of the initial grid, else 1.
                                  The 4-wide walk and a batch always share */
    double super_fraction;     /* size of the super-box table (one entry per aligned 2x2x2 block of boxes) per
                                  simulation, as a fraction of its box capacity: 0 (default) = enough for any
                                  grid of box_capacity boxes, ceil((capacity + 1) / 2) entries (a grid one box
                                  thick); f in (0, 1] = min(that, ceil(f * capacity) + 64) entries, about
                                  capacity / 8 for grids of many boxes along each axis.  A grid with more
                                  super-boxes fails like one above the box capacity (ABM_E_GRID).  Fixed at
                                  init; a batch takes per_sim[0]'s */
} abm_params;

/* Grid extent of a set of positions (Section 3.1), as abm_extent reports it. */
typedef struct abm_extent {
    double radius;             /* interaction radius R */
    double inv_cell;           /* 1 / (cell_factor * R), evaluated in double */
    int64_t cmin[3];           /* smallest box coordinate floor(x * inv_cell) per axis */
    int64_t dims[3];           /* boxes per axis */
    int64_t nboxes;            /* dims[0] * dims[1] * dims[2] */
} abm_extent;

/* Per-step statistics of the last completed step (Section 5's engine tracks
 * which agents moved and which were skipped). */
typedef struct abm_stats {
    int64_t step;              /* steps completed */
    int64_t n_static;          /* agents whose force was skipped */
    int64_t n_moved;           /* agents with a non-zero displacement */
    uint32_t error;            /* device error bits (0 = none) */
    uint32_t build;            /* the last step's grid: bit 0 set for an update of the grid before (Section 3.1's
                                  grid kept, only the super-boxes agents entered or left rebuilt), clear for a full
                                  build; bits 1..31 the simulations of a batch rebuilt inside that update (their
                                  extent changed) */
    double sum_force[3];       /* sum of the forces the step evaluated (every agent's with the static test off:
                                  zero up to rounding by Newton's third law, each pair term entering twice with
                                  opposite signs); summed in a fixed order for a single simulation */
    double max_displacement;   /* largest |Delta_i| of the step: |mu F_i|, or delta_max where clamped */
    double skip_fraction;      /* n_static / n */
} abm_stats;

/* Accumulated kernel times of timed steps (abm_set_timing / abm_get_timing):
 * ms[0] setup, ms[1] box keys + histogram, ms[2] scan, ms[3] scatter,
 * ms[4] canonical order + box table, ms[5] static flags + force + move;
 * ms[6], ms[7] unused (0). */
typedef struct abm_timing {
    int64_t steps;
    double ms[8];
} abm_timing;

typedef struct abm_ctx abm_ctx;

/* Fields for abm_query. */
enum abm_field {
    ABM_FIELD_POSITIONS = 0,   /* n x 3 element type, by agent id */
    ABM_FIELD_FORCES = 1,      /* n x 3 double, by agent id (needs keep_forces) */
    ABM_FIELD_MOVED = 2,       /* n uint8, by agent id: displacement of the last step was non-zero */
    ABM_FIELD_STATIC = 3,      /* n uint8, by agent id: the force was skipped in the last step */
    ABM_FIELD_NNZ = 4,         /* n int32, by agent id: non-zero pair terms in the last force evaluation */
    ABM_FIELD_KEY = 5,         /* n uint32, by agent id: gap-free rank of the agent's box in the context's order
                                  (last grid) */
    ABM_FIELD_PERM = 6,        /* n uint32: agent ids in (box rank, id) order of the last grid */
    ABM_FIELD_CELL_START = 7,  /* nboxes + 1 uint32: first slot of each box, last grid (single simulation;
                                  ABM_E_UNSUPPORTED for a batched context) */
    ABM_FIELD_EXTENT = 8,      /* int64[7] per simulation: cmin[3], dims[3], nboxes of the last grid */
    ABM_FIELD_STORAGE_IDS = 9, /* n uint32: agent id held by each storage slot */
    ABM_FIELD_NEIGHBOR_COUNT = 10, /* n uint32, by agent id: |N(i)| = #{j != i : |x_i - x_j|^2 < R^2} on the
                                      positions of the last grid (Section 3.1's neighbourhood) */
    ABM_FIELD_NEIGHBORS = 11,  /* n x K uint32, by agent id, K = dst_bytes / (4 n): the ids of N(i) in
                                  ascending order, padded with 0xFFFFFFFF; ABM_E_INVAL if some |N(i)| > K */
    ABM_FIELD_DIAMETERS = 12   /* n element type, by agent id */
};

/* Version of this ABI (ABM_ABI_VERSION). */
int abm_abi_version(void);

/* Fill *p with the defaults listed in abm_params. */
void abm_default_params(abm_params* p);

/* Message for the last failure on the calling thread ("" if none). */
const char* abm_last_error(void);

/*
 * Grid extent of n agents (Section 3.1: box = floor(x / edge) per axis).
 * pos, diam: device, element type per p->precision.  scratch: device, at
 * least ABM_EXTENT_SCRATCH_BYTES bytes, 8-byte aligned, caller-owned,
 * clobbered.  Synchronises `stream`.  Errors: ABM_E_INVAL, ABM_E_NONFINITE,
 * ABM_E_HIP.
 */
int abm_extent_of(int64_t n, const void* pos, const void* diam, const abm_params* p, void* scratch,
                  void* stream, abm_extent* out);

/*
 * abm_extent_of for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, with the scratch taken from a fixed array of
 * ABM_EXTENT_SCRATCH_BYTES (1 KiB) in the library's own device memory, one
 * copy per GPU, held until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); its first call on a
 * device looks up that device's copy.  Every call on one GPU shares that
 * copy: calls that overlap on one GPU (other host threads, other streams)
 * race and must be serialised by the caller.  The scratch need does not grow
 * with n; n above ABM_NOALLOC_MAX_AGENTS is refused with ABM_E_INVAL.
 * Synchronises `stream`.  Errors: ABM_E_INVAL, ABM_E_NONFINITE, ABM_E_HIP,
 * ABM_E_UNSUPPORTED (device index above 63).
 */
#define ABM_NOALLOC_MAX_AGENTS 4294967294LL
int abm_extent_of_noalloc(int64_t n, const void* pos, const void* diam, const abm_params* p, void* stream,
                          abm_extent* out);

/*
 * Bytes of device workspace for nsims simulations with the given agent
 * offsets (host, nsims + 1, offsets[0] = 0; at most 2^31 - 2^20 agents in
 * all) and box capacities (host, nsims: boxes each simulation's grid may
 * span; see abm_extent.nboxes).  The per-box tables are held per super-box,
 * ceil((capacity + 1) / 2) entries per simulation, or fewer with
 * p->super_fraction (which the workspace of a context must have been sized
 * with).
 */
int abm_workspace_bytes(int32_t nsims, const int64_t* offsets, const int64_t* box_capacity,
                        const abm_params* p, int64_t* bytes);

/*
 * Create a context for one simulation of n agents (Algorithm 1's model
 * initialisation).  pos (n x 3) and diam (n): device, element type per
 * p->precision, copied at init.  box_capacity: largest number of grid boxes
 * the run may need (>= the initial abm_extent.nboxes).  ws: device
 * workspace of ws_bytes >= abm_workspace_bytes(), 256-byte aligned, kept until
 * abm_destroy.  Agent ids are 0..n-1 in input order; at step 0 every agent
 * counts as moved, so none is static.  Errors: ABM_E_INVAL, ABM_E_WORKSPACE,
 * ABM_E_NONFINITE (diameters not finite and > 0), ABM_E_HIP.
 */
int abm_init(abm_ctx** ctx, int64_t n, const void* pos, const void* diam, const abm_params* p,
             int64_t box_capacity, void* ws, int64_t ws_bytes, void* stream);

/*
 * Batched form: nsims independent simulations in one context.  offsets
 * (host, nsims + 1) delimit each simulation's agents in pos/diam; per_sim
 * (host, nsims) gives each simulation's parameters (precision, sort_every,
 * block_size, keep_forces and detect_static are taken from per_sim[0]);
 * box_capacity (host, nsims).  Agent ids are global input indices.  Each
 * simulation advances exactly as it would alone.  Each simulation owns a
 * fixed range of the super-box table (ceil((capacity + 1) / 2) entries, or
 * per_sim[0].super_fraction of its capacity + 64), scanned every step; a
 * step's grid is an update of the last one in which the simulations whose
 * extent changed are rebuilt (a full build when a quarter of the agents or
 * more belong to them; abm_stats.build reports which).
 */
int abm_init_batched(abm_ctx** ctx, int32_t nsims, const int64_t* offsets, const void* pos, const void* diam,
                     const abm_params* per_sim, const int64_t* box_capacity, void* ws, int64_t ws_bytes,
                     void* stream);

/*
 * Dynamic population (Section 3.2: agents are added and removed between
 * iterations).  abm_workspace_bytes_capacity gives the workspace of a
 * single-simulation context that holds up to `capacity` agents (1 <= capacity
 * <= 2^31 - 2^20); abm_init_capacity creates one with n <= capacity agents,
 * otherwise as abm_init.  The interaction radius stays the one fixed at init
 * (the largest initial diameter unless p->interaction_radius > 0).
 */
int abm_workspace_bytes_capacity(int64_t capacity, int64_t box_capacity, const abm_params* p, int64_t* bytes);
int abm_init_capacity(abm_ctx** ctx, int64_t n, int64_t capacity, const void* pos, const void* diam,
                      const abm_params* p, int64_t box_capacity, void* ws, int64_t ws_bytes, void* stream);

/*
 * Append m agents between steps (Section 3.2): pos (m x 3) and diam (m) on
 * the device, element type of the context, read before the call returns.
 * They get ids n, n+1, ..., n+m-1, count as moved in the last step (no
 * history; so no agent within R of one is static in the next step, condition
 * (iii) of Section 5), with no pair terms and no force.  The call
 * synchronizes the context's stream.  Errors: ABM_E_INVAL (n + m above the
 * capacity, or a diameter above the interaction radius: the population is
 * then unchanged), ABM_E_NONFINITE, ABM_E_UNSUPPORTED (batched context).
 */
int abm_add_agents(abm_ctx* ctx, int64_t m, const void* pos, const void* diam);

/*
 * Remove the m agents with the given ids (device, m distinct int64 ids below
 * n) between steps, keeping the ids dense as Section 3.2 keeps the agent
 * vector dense: with new_size = n - m, each removed id below new_size is a
 * hole that a kept id at or above new_size takes over, the k-th hole in
 * ascending order the k-th such id in ascending order; every other agent
 * keeps its id.  Agents near a removed one keep their static state
 * (condition (iv) of Section 5).  The call synchronizes the context's stream.
 * Errors: ABM_E_INVAL (an id out of range or given twice, or m = n: nothing
 * is removed then), ABM_E_UNSUPPORTED (batched context).
 */
int abm_remove_agents(abm_ctx* ctx, int64_t m, const int64_t* ids);

/*
 * Give the m agents with the given ids (device, m distinct int64 ids below n)
 * the diameters diam (device, m values of the context's element type) between
 * steps: growth, shrinking, or the mother's half of a division (whose
 * daughter abm_add_agents appends).  Condition (ii) of Section 5: an agent
 * whose diameter changed counts as moved in the last step, so neither it nor
 * an agent within R of it is static in the next step; under this force law a
 * smaller diameter can raise a pair force as well as a larger one.  An
 * unchanged value changes nothing.  Positions and boxes stay, so the last
 * grid and a captured graph remain valid; a recorded forward run does not.
 * Works for batched contexts (ids are global agent indices).  The call reads
 * its inputs and synchronizes the context's stream before it returns.
 * Errors (nothing changes then): ABM_E_INVAL (an id out of range or given
 * twice, or a diameter above the interaction radius of its simulation),
 * ABM_E_NONFINITE (a diameter not finite and > 0).
 */
int abm_set_diameters(abm_ctx* ctx, int64_t m, const int64_t* ids, const void* diam);

/* Agents now and the context's capacity (host outputs; either may be null). */
int abm_population(abm_ctx* ctx, int64_t* n, int64_t* capacity);

/*
 * Change the force-law, mobility, threshold or clamp parameters (all
 * simulations of a batched context take the same values).  Every agent counts
 * as moved at the next step, so none is static there (Section 5: a changed
 * attribute unsets static agents).
 */
int abm_set_params(abm_ctx* ctx, const abm_params* p);

/*
 * Enqueue nsteps steps (Algorithm 1's iteration loop): grid build, static
 * flags, forces, displacement.  Asynchronous; device-detected errors (grid
 * overflow, non-finite positions) are reported by the next abm_sync/query.
 */
int abm_step(abm_ctx* ctx, int32_t nsteps);

/* Wait for the stream; returns the first device error as ABM_E_* (cleared). */
int abm_sync(abm_ctx* ctx);

/*
 * Copy a field (enum abm_field) into dst (device if dst_is_device, else
 * host) of dst_bytes.  Synchronises the stream.
 */
int abm_query(abm_ctx* ctx, int32_t field, void* dst, int64_t dst_bytes, int32_t dst_is_device);

/* Statistics of the last completed step (synchronises). */
int abm_get_stats(abm_ctx* ctx, abm_stats* out);

/*
 * Checkpoint / resume: abm_state_bytes gives the size; export writes
 * positions, moved flags, non-zero counts and the step counter to host
 * memory; import restores them into a context of the same shape.
 */
int abm_state_bytes(abm_ctx* ctx, int64_t* bytes);
int abm_export_state(abm_ctx* ctx, void* dst, int64_t dst_bytes);
int abm_import_state(abm_ctx* ctx, const void* src, int64_t src_bytes);

/*
 * Capture nsteps steps into one HIP graph (replaces any earlier graph) and
 * replay it with abm_graph_launch; a replay advances the context by nsteps.
 * The context's stream must not be the null stream.  nsteps must be even and
 * a multiple of sort_every, so that every replay starts from the same
 * internal buffers.  Errors: ABM_E_INVAL, ABM_E_HIP; abm_graph_launch
 * without a graph: ABM_E_STATE.
 */
int abm_graph_capture(abm_ctx* ctx, int32_t nsteps);
int abm_graph_launch(abm_ctx* ctx);

/*
 * Reverse mode of the step x -> x + Delta(F(x); k, gamma) with the neighbour
 * sets, thresholds and clamp states of every forward step held fixed
 * (single simulation, detect_static off).
 *   abm_record_sizes: device bytes of a record of nsteps with a checkpoint
 *     every ckpt_every steps, in three sizes (sizes: host, 3 int64):
 *     sizes[0] the least; sizes[1] with room for one segment's contact tapes;
 *     sizes[2] with room for every step's tapes.  abm_record_bytes gives
 *     sizes[2].  A contact tape holds every agent's contacts on one step's
 *     grid, in the order the force sums them (32 per agent at most); a
 *     reverse step that reads a complete tape needs no grid and no
 *     neighbour walk, and gives the same result, bit for bit.
 *   abm_forward_record: run nsteps steps from the current state (re-laying
 *     agents out every sort_every steps, as abm_step does), keeping the
 *     positions of every ckpt_every-th step in rec (device, rec_bytes of at
 *     least sizes[0], 256-byte aligned; the caller owns it and keeps it
 *     until the backward is done).  With rec_bytes >= sizes[2] it also tapes
 *     every step, and the backward recomputes nothing unless a tape is
 *     incomplete (an agent with more than 32 contacts).
 *   abm_backward: given dL/dx_T (device, n x 3 double, by id), write
 *     dL/dx_0 (device, n x 3 double, by id) and dL/d(k, gamma) (device,
 *     2 double).  Without complete tapes of every step it recomputes each
 *     checkpoint segment forward (taping its steps if rec_bytes >=
 *     sizes[1]), then walks it backward, on the tape of each step whose tape
 *     is complete and else on a grid built from the step's positions.
 *     ABM_E_STATE without a preceding abm_forward_record.
 *   abm_record_info: info (host, 3 int32): [0] the record's tapes (-1 no
 *     record, 0 none, 1 per recomputed segment, 2 every step); [1] reverse
 *     steps of the last abm_backward that read a tape; [2] the largest
 *     contact count a tape has seen.
 */
int abm_record_bytes(abm_ctx* ctx, int32_t nsteps, int32_t ckpt_every, int64_t* bytes);
int abm_record_sizes(abm_ctx* ctx, int32_t nsteps, int32_t ckpt_every, int64_t* sizes);
int abm_forward_record(abm_ctx* ctx, int32_t nsteps, int32_t ckpt_every, void* rec, int64_t rec_bytes);
int abm_backward(abm_ctx* ctx, const void* dL_dxT, void* dL_dx0, void* dL_dparams);
int abm_record_info(abm_ctx* ctx, int32_t* info);

/*
 * Timing mode: with enable = 1, every step enqueued by abm_step brackets
 * each of its kernels with HIP events on the context's stream; with
 * enable = 2, only the static flags + force + move kernel (ms[5]; the other
 * entries stay 0), which adds fewer events to the steps; 0 turns timing off
 * (graph replays are not timed).  abm_set_timing resets the accumulators;
 * abm_get_timing synchronises and adds the elapsed times of all timed steps
 * so far.
 */
int abm_set_timing(abm_ctx* ctx, int32_t enable);
int abm_get_timing(abm_ctx* ctx, abm_timing* out);

/* Release the context (not the caller's buffers). */
void abm_destroy(abm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ABM_H */
