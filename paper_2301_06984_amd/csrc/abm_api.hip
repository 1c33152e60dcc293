// abm_api.hip -- the C ABI of libabm (declared in include/abm.h): workspace
// layout, step sequencing (Algorithm 1's iteration as a chain of kernels on
// one stream), queries, checkpoints, graph capture and the adjoint driver.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/abm.h"
#include "abm_internal.h"

using namespace abm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(ABM_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// setup, keys, scan, scatter, fixup, force
constexpr int kTimedPhases = 6;

struct Layout {
    int64_t globals, sims, sim_of, bbox_rep, pos4[2], flags[2], skey[2], ids[2], force[2], key, sub, rec, perm, movers,
        mcount, count, cell_start[2], dirty, dirty_list, aoff, tabidx, mmask, cellinfo, hil, tile_sums, partials,
        bpart, stage, total;
    uint32_t scan_tiles, partial_cap, bpart_cap;
};

// Agents per context: loose slots [0, 2n) and the padded step grid stay below 2^32.
constexpr int64_t kMaxAgents = (int64_t(1) << 31) - (int64_t(1) << 20);

// Super-boxes of a grid of at most cap boxes: prod ceil(d_a / 2) with d_x d_y
// d_z <= cap is largest for dims (1, 1, cap), so at most ceil((cap + 1) / 2);
// with a fraction f > 0 the table holds min(that, ceil(f cap) + 64) entries
// (a grid with more super-boxes is refused at setup, as one above the box
// capacity).
int64_t super_capacity(int64_t cap, double f) {
    const int64_t any = (cap + 2) / 2;
    if (!(f > 0.0)) return any;
    const int64_t t = int64_t(std::ceil(f * double(cap))) + 64;
    return t < any ? t : any;
}

// boxes: capacity in super-boxes (sum of super_capacity over the simulations)
Layout make_layout(int64_t n, int32_t nsims, int64_t boxes, bool keep_forces, int64_t elem) {
    Layout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.globals = take(sizeof(Globals));
    L.sims = take(int64_t(sizeof(SimGrid)) * nsims);
    L.sim_of = nsims > 1 ? take(2 * n) : -1;
    L.bbox_rep = take(int64_t(sizeof(int32_t)) * 2 * kReplicas * nsims * 6);
    // loose slots [0, 2n) of the grid, positions padded for the walk
    for (int k = 0; k < 2; ++k) L.pos4[k] = take(4 * elem * (2 * n + kSposPad));
    for (int k = 0; k < 2; ++k) L.flags[k] = take(4 * 2 * n);
    for (int k = 0; k < 2; ++k) L.skey[k] = take(4 * 2 * n);
    for (int k = 0; k < 2; ++k) L.ids[k] = take(4 * n);
    for (int k = 0; k < 2; ++k) L.force[k] = keep_forces ? take(24 * n) : -1;
    L.key = take(4 * n);
    L.sub = take(4 * n);
    L.rec = take(16 * n);
    L.perm = take(4 * n);
    L.movers = take(4 * n);
    L.mcount = take(4 * ((n + 255) / 256));
    L.count = take(4 * boxes);
    for (int k = 0; k < 2; ++k) L.cell_start[k] = take(4 * (boxes + 1));
    L.dirty = take(4 * boxes);
    L.dirty_list = take(4 * boxes);
    L.aoff = take(4 * boxes);
    L.tabidx = take(4 * boxes);
    L.mmask = take(4 * boxes);
    L.cellinfo = take(16 * boxes);
    L.hil = take(sizeof(HilbertTables));
    L.scan_tiles = uint32_t((boxes + kScanTile - 1) / kScanTile);
    if (L.scan_tiles == 0) L.scan_tiles = 1;
    L.tile_sums = take(12 * int64_t(L.scan_tiles));
    L.partial_cap = uint32_t(adj_blocks(uint32_t(n)));
    L.partials = take(16 * int64_t(L.partial_cap));
    L.bpart_cap = force_part_capacity(uint32_t(n));
    L.bpart = take(int64_t(sizeof(BlockPart)) * L.bpart_cap);
    // staging for the host calls between steps: key, sub and rec (contiguous,
    // 24 B per agent and more with the alignment), which only a grid build uses
    L.stage = L.key;
    L.total = off;
    return L;
}

}  // namespace

struct abm_ctx {
    int precision = ABM_F32;
    int32_t nsims = 1;
    int64_t n = 0;           // agents now
    int64_t cap = 0;         // agents the workspace holds (additions up to it)
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L{};
    Buffers<float> bf{};
    Buffers<double> bd{};
    std::vector<int64_t> offsets;
    abm_params params{};
    int walk_chunk = 2;      // candidates the neighbour walk tests together (2 or 4)
    bool share = false;      // the 2-wide walk of one simulation shares out the wave's pair terms
    int cs_cur = 0;          // which cell_start copy the next grid build writes (the other holds the last)
    bool inc_ready = false;  // agents are stored in the last grid's canonical order, positions from the step
    bool graph_inc_after = false;
    int grid_pos = 0;        // pos4/skey copy holding the last grid's loose slots
    // host mirror of the device state
    int64_t step = 0;
    int pos_cur = 0;
    int ids_cur = 0;
    int grid_ids = 0;        // ids buffer that the last grid's key/perm refer to
    bool have_grid = false;
    uint32_t stamp_count = 0;  // device stamp value after the last enqueued step
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int32_t graph_steps = 0;
    int graph_grid_ids = 0;  // ids buffer of the last captured step's grid
    // timing mode: 0 off; 1 one set of events per step around each kernel;
    // 2 events around the step kernel only
    int timing = 0;
    std::vector<std::array<hipEvent_t, kTimedPhases + 1>> ev_pending, ev_free;
    double ev_ms[kTimedPhases] = {};
    int64_t ev_steps = 0;
    // adjoint record
    bool recorded = false;
    int32_t rec_steps = 0, rec_ckpt = 0;
    int64_t rec_start = 0;
    char* rec = nullptr;
    int64_t rec_bytes = 0;
    // contact tapes of the record: 0 none (the reverse steps walk a grid), 1
    // written per segment while it is recomputed, 2 written by the record for
    // every step (no recomputation)
    int rec_tapes = 0;
    uint32_t rec_worst = 0;        // the largest contact count a tape saw
    int32_t taped_reverse = 0;     // reverse steps of the last backward that read a tape
    TapeStep tape_next{};          // the next step's grid is taped here (pos null: not taped)

    int64_t elem() const { return precision == ABM_F64 ? 8 : 4; }
    template <class T> Buffers<T>& buf();
};
template <> Buffers<float>& abm_ctx::buf<float>() { return bf; }
template <> Buffers<double>& abm_ctx::buf<double>() { return bd; }

namespace {

template <class T>
void fill_buffers(abm_ctx* c) {
    Buffers<T>& b = c->buf<T>();
    char* w = c->ws;
    const Layout& L = c->L;
    b.g = reinterpret_cast<Globals*>(w + L.globals);
    b.sims = reinterpret_cast<SimGrid*>(w + L.sims);
    b.sim_of = L.sim_of >= 0 ? reinterpret_cast<const uint16_t*>(w + L.sim_of) : nullptr;
    b.bbox_rep = reinterpret_cast<int32_t*>(w + L.bbox_rep);
    b.nsims = c->nsims;
    b.n = uint32_t(c->n);
    for (int k = 0; k < 2; ++k) {
        b.pos4[k] = w + L.pos4[k];
        b.flags[k] = reinterpret_cast<uint32_t*>(w + L.flags[k]);
        b.skey[k] = reinterpret_cast<uint32_t*>(w + L.skey[k]);
        b.ids[k] = reinterpret_cast<uint32_t*>(w + L.ids[k]);
        b.force[k] = L.force[k] >= 0 ? reinterpret_cast<double*>(w + L.force[k]) : nullptr;
    }
    b.key = reinterpret_cast<uint32_t*>(w + L.key);
    b.sub = reinterpret_cast<uint32_t*>(w + L.sub);
    b.rec = reinterpret_cast<uint4*>(w + L.rec);
    b.perm = reinterpret_cast<uint32_t*>(w + L.perm);
    b.movers = reinterpret_cast<uint32_t*>(w + L.movers);
    b.mcount = reinterpret_cast<uint32_t*>(w + L.mcount);
    b.gpos = b.pos4[c->grid_pos];
    b.gkey = b.skey[c->grid_pos];
    b.count = reinterpret_cast<uint32_t*>(w + L.count);
    b.cell_start = reinterpret_cast<uint32_t*>(w + L.cell_start[c->cs_cur]);
    b.cell_start_old = reinterpret_cast<uint32_t*>(w + L.cell_start[c->cs_cur ^ 1]);
    b.dirty = reinterpret_cast<uint32_t*>(w + L.dirty);

    b.dirty_list = reinterpret_cast<uint32_t*>(w + L.dirty_list);
    b.aoff = reinterpret_cast<uint32_t*>(w + L.aoff);
    b.tabidx = reinterpret_cast<uint32_t*>(w + L.tabidx);
    b.mmask = reinterpret_cast<uint32_t*>(w + L.mmask);
    b.cellinfo = reinterpret_cast<uint4*>(w + L.cellinfo);
    b.hil = c->params.order == ABM_ORDER_HILBERT ? reinterpret_cast<const HilbertTables*>(w + L.hil) : nullptr;
    b.tile_sums = reinterpret_cast<uint32_t*>(w + L.tile_sums);
    b.scan_tiles = L.scan_tiles;
    b.partials = reinterpret_cast<double*>(w + L.partials);
    b.partial_cap = L.partial_cap;
    b.bpart = reinterpret_cast<BlockPart*>(w + L.bpart);
    b.bpart_cap = L.bpart_cap;
}

// After a grid build: its starts become the last grid's.
template <class T>
void swap_cell_start(abm_ctx* c) {
    c->cs_cur ^= 1;
    Buffers<T>& b = c->buf<T>();
    b.cell_start = reinterpret_cast<uint32_t*>(c->ws + c->L.cell_start[c->cs_cur]);
    b.cell_start_old = reinterpret_cast<uint32_t*>(c->ws + c->L.cell_start[c->cs_cur ^ 1]);
}

// The grid about to be built (and then queried) holds its loose slots in
// pos4/skey copy `pos`.
template <class T>
void set_grid_pos(abm_ctx* c, int pos) {
    c->grid_pos = pos;
    Buffers<T>& b = c->buf<T>();
    b.gpos = b.pos4[pos];
    b.gkey = b.skey[pos];
}

// Super-box starts of the last grid (after its build swapped the copies).
template <class T>
const uint32_t* last_grid_starts(abm_ctx* c) {
    return reinterpret_cast<const uint32_t*>(c->ws + c->L.cell_start[c->cs_cur ^ 1]);
}

// The Hilbert order's tables, built on first use and kept for the process
// (the same for every context; null if they cannot be built).
const HilbertTables* hilbert_tables() {
    static HilbertTables t;
    static const bool ok = build_hilbert_tables(&t);
    return ok ? &t : nullptr;
}

bool valid_params(const abm_params* p, std::string* why) {
    if (!p) return *why = "params is null", false;
    if (p->precision != ABM_F32 && p->precision != ABM_F64) return *why = "precision must be ABM_F32 or ABM_F64", false;
    const double v[] = {p->k, p->gamma, p->mu, p->f_adh, p->delta_max, p->interaction_radius, p->cell_factor};
    for (double x : v)
        if (!std::isfinite(x)) return *why = "non-finite parameter", false;
    if (p->delta_max < 0 || p->mu < 0 || p->interaction_radius < 0)
        return *why = "mu, delta_max and interaction_radius must be >= 0", false;
    if (p->cell_factor < 1.0) return *why = "cell_factor must be >= 1", false;
    if (p->sort_every < 0) return *why = "sort_every must be >= 0", false;
    if (p->block_size != 0 && (p->block_size < 64 || p->block_size > 1024 || p->block_size % 64))
        return *why = "block_size must be 0 or a multiple of 64 in [64, 1024]", false;
    if (p->walk_chunk != 0 && p->walk_chunk != 2 && p->walk_chunk != 4)
        return *why = "walk_chunk must be 0, 2 or 4", false;
    if (p->share_terms < 0 || p->share_terms > 2) return *why = "share_terms must be 0, 1 or 2", false;
    if (p->order != ABM_ORDER_MORTON && p->order != ABM_ORDER_HILBERT)
        return *why = "order must be ABM_ORDER_MORTON or ABM_ORDER_HILBERT", false;
    if (!(p->super_fraction >= 0.0 && p->super_fraction <= 1.0))
        return *why = "super_fraction must be in [0, 1]", false;
    return true;
}

int block_size_of(const abm_params& p) { return p.block_size ? p.block_size : 256; }

// Decode the device error word into a status code.
int error_code(uint32_t err) {
    if (err & kErrNonfinite) return fail(ABM_E_NONFINITE, "non-finite position or diameter");
    if (err & kErrGrid) return fail(ABM_E_GRID, "grid exceeds its box capacity or 2^21 boxes per axis");
    if (err & kErrRange)
        return fail(ABM_E_INVAL, "value out of range (an added diameter above the interaction radius, or an id "
                                 "out of range or given twice)");
    if (err & kErrInternal) return fail(ABM_E_HIP, "internal index check failed");
    return ABM_OK;
}

int read_error(abm_ctx* c, bool clear) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    uint32_t err = 0;
    Globals* g = reinterpret_cast<Globals*>(c->ws + c->L.globals);
    HIP_TRY(hipMemcpy(&err, &g->err, sizeof(err), hipMemcpyDeviceToHost));
    if (err && clear) HIP_TRY(hipMemset(&g->err, 0, sizeof(err)));
    return error_code(err);
}

template <class T>
void enqueue_extent(abm_ctx* c) {
    const int parity = int(c->step & 1);
    launch_bbox<T>(c->buf<T>(), c->pos_cur, parity, c->stream);
}

// Clear the box table and restart the stamps if m more steps would wrap them.
template <class T>
void guard_stamps(abm_ctx* c, int64_t m) {
    if (int64_t(c->stamp_count) + m > int64_t(kStampPeriod)) {
        launch_clear_cellinfo<T>(c->buf<T>(), c->stream);
        c->stamp_count = 0;
        c->inc_ready = false;   // an update build reuses the table entries
    }
}

std::array<hipEvent_t, kTimedPhases + 1>* next_events(abm_ctx* c) {
    if (c->ev_free.empty()) {
        std::array<hipEvent_t, kTimedPhases + 1> e{};
        for (auto& x : e)
            if (hipEventCreate(&x) != hipSuccess) return nullptr;
        c->ev_free.push_back(e);
    }
    c->ev_pending.push_back(c->ev_free.back());
    c->ev_free.pop_back();
    return &c->ev_pending.back();
}

template <class T>
void enqueue_step(abm_ctx* c, bool allow_relayout, int timed = 0) {
    Buffers<T>& b = c->buf<T>();
    const int parity = int(c->step & 1);
    std::array<hipEvent_t, kTimedPhases + 1>* ev = timed ? next_events(c) : nullptr;
    const bool all_phases = ev && timed == 1;
    hipEvent_t* marks[4] = {nullptr, nullptr, nullptr, nullptr};
    if (all_phases) {
        (void)hipEventRecord((*ev)[0], c->stream);
        for (int k = 0; k < 4; ++k) marks[k] = &(*ev)[2 + k];
    }
    StepArgs a{};
    a.parity = parity;
    a.pos_cur = c->pos_cur;
    a.ids_cur = c->ids_cur;
    a.relayout = allow_relayout && c->params.sort_every > 0 && ((c->step + 1) % c->params.sort_every == 0);
    a.detect_static = c->params.detect_static != 0;
    a.keep_forces = c->params.keep_forces != 0;
    a.block_size = block_size_of(c->params);
    a.walk_chunk = c->walk_chunk;
    a.share = c->share;
    a.full_only = !c->inc_ready;
    set_grid_pos<T>(c, c->pos_cur);
    launch_setup<T>(b, parity, c->inc_ready, c->stream);
    if (all_phases) (void)hipEventRecord((*ev)[1], c->stream);
    launch_grid<T>(b, c->pos_cur, c->ids_cur, a.relayout, a.detect_static, c->stream, all_phases ? marks : nullptr);
    swap_cell_start<T>(c);
    a.cs = last_grid_starts<T>(c);
    if (c->tape_next.pos) {
        // the step kernel tapes a full build of one simulation without the
        // static test (every step the adjoint records)
        if (c->nsims == 1 && !a.detect_static && a.full_only)
            a.tape = c->tape_next;
        else
            launch_adj_tape<T>(b, c->ids_cur, c->tape_next, c->stream);
        c->tape_next = TapeStep{};
    }
    if (ev && !all_phases) (void)hipEventRecord((*ev)[kTimedPhases - 1], c->stream);
    launch_force<T>(b, a, c->stream);
    if (ev) (void)hipEventRecord((*ev)[kTimedPhases], c->stream);
    c->grid_ids = c->ids_cur;
    c->have_grid = true;
    c->pos_cur ^= 1;
    if (a.relayout) c->ids_cur ^= 1;
    // after a re-layout the agents are stored in this grid's canonical order,
    // so the next grid can be built as an update of this one
    c->inc_ready = a.relayout;
    c->step += 1;
    c->stamp_count += 1;
}

template <class T>
int do_steps(abm_ctx* c, int32_t nsteps, bool allow_relayout) {
    int32_t left = nsteps;
    while (left > 0) {
        const int32_t m = left < int32_t(kStampPeriod) ? left : int32_t(kStampPeriod);
        guard_stamps<T>(c, m);
        for (int32_t s = 0; s < m; ++s) enqueue_step<T>(c, allow_relayout, c->timing);
        left -= m;
    }
    HIP_TRY(hipGetLastError());
    return ABM_OK;
}

int check_ctx(abm_ctx* c) {
    if (!c || !c->ws) return fail(ABM_E_INVAL, "null or destroyed context");
    return ABM_OK;
}

template <class T>
int init_impl(abm_ctx** out, int32_t nsims, const int64_t* offsets, const void* pos, const void* diam,
              const abm_params* per_sim, const int64_t* box_capacity, void* ws, int64_t ws_bytes, void* stream,
              int64_t capacity) {
    const int64_t n = offsets[nsims];
    const int64_t cap = std::max(capacity, n);
    // loose slots [0, 2n) and the padded step grid stay below 2^32
    if (cap > kMaxAgents) return fail(ABM_E_INVAL, "at most 2^31 - 2^20 agents");
    std::vector<SimGrid> sims(nsims);
    uint64_t boxes = 0, supers = 0;
    for (int s = 0; s < nsims; ++s) {
        std::string why;
        if (!valid_params(&per_sim[s], &why)) return fail(ABM_E_INVAL, "simulation " + std::to_string(s) + ": " + why);
        if (offsets[s + 1] <= offsets[s]) return fail(ABM_E_INVAL, "every simulation needs at least one agent");
        if (per_sim[s].order != per_sim[0].order) return fail(ABM_E_INVAL, "all simulations need the same order");
        if (box_capacity[s] < 1 || box_capacity[s] > 0xFFFFFFFFll)
            return fail(ABM_E_INVAL, "box capacity must be in [1, 2^32)");
        boxes += uint64_t(box_capacity[s]);
        const uint64_t scap = uint64_t(super_capacity(box_capacity[s], per_sim[0].super_fraction));
        SimGrid& G = sims[s];
        std::memset(&G, 0, sizeof(G));
        // several simulations: each owns a fixed range of the super-box table
        G.sbase = nsims > 1 ? uint32_t(supers) : 0u;
        G.scap = uint32_t(scap);
        supers += scap;
        G.radius = per_sim[s].interaction_radius;
        G.k = per_sim[s].k;
        G.gamma = per_sim[s].gamma;
        G.mu = per_sim[s].mu;
        G.f_adh = per_sim[s].f_adh;
        G.delta_max = per_sim[s].delta_max;
        G.cell_factor = per_sim[s].cell_factor;
        G.agent_begin = uint32_t(offsets[s]);
        G.agent_end = uint32_t(offsets[s + 1]);
        G.cap = uint32_t(box_capacity[s]);
    }
    if (boxes >= 0xFFFFFFFFull) return fail(ABM_E_GRID, "total box capacity must be below 2^32");
    if (nsims > 1 && supers >= uint64_t(kMaxSuperBoxes))
        return fail(ABM_E_GRID, "the simulations' super-box capacities must sum below 2^29");
    const abm_params& p0 = per_sim[0];
    const Layout L = make_layout(cap, nsims, int64_t(supers), p0.keep_forces != 0, sizeof(T));
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return fail(ABM_E_INVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(ABM_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");
    abm_ctx* c = new abm_ctx();
    c->precision = p0.precision;
    c->nsims = nsims;
    c->n = n;
    c->cap = cap;
    c->stream = static_cast<hipStream_t>(stream);
    c->ws = static_cast<char*>(ws);
    c->L = L;
    c->offsets.assign(offsets, offsets + nsims + 1);
    c->params = p0;
    fill_buffers<T>(c);
    Buffers<T>& b = c->buf<T>();
    b.super_capacity = uint32_t(supers);
    hipStream_t s = c->stream;
    auto bail = [&](int code) {
        delete c;
        return code;
    };
    // zero what must start at zero: globals, histogram, box table, change
    // marks, table indices, moved masks; and the positions with their padding (read,
    // never used, by the walk)
    if (hipMemsetAsync(c->ws + L.globals, 0, sizeof(Globals), s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.count, 0, 4 * supers, s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.cellinfo, 0, 16 * supers, s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.dirty, 0, 4 * supers, s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.tabidx, 0, 4 * supers, s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.mmask, 0, 4 * supers, s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.pos4[0], 0, 4 * c->elem() * (2 * cap + kSposPad), s) != hipSuccess ||
        hipMemsetAsync(c->ws + L.pos4[1], 0, 4 * c->elem() * (2 * cap + kSposPad), s) != hipSuccess ||
        hipMemcpyAsync(b.sims, sims.data(), sizeof(SimGrid) * nsims, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(ABM_E_HIP, "workspace initialisation failed"));
    if (b.hil) {
        const HilbertTables* t = hilbert_tables();
        if (!t) return bail(fail(ABM_E_HIP, "the Hilbert curve's tables could not be built"));
        if (hipMemcpyAsync(c->ws + L.hil, t, sizeof(HilbertTables), hipMemcpyHostToDevice, s) != hipSuccess)
            return bail(fail(ABM_E_HIP, "Hilbert table upload failed"));
    }
    std::vector<uint16_t> sim_of;
    if (nsims > 1) {
        sim_of.resize(n);
        for (int q = 0; q < nsims; ++q)
            for (int64_t i = offsets[q]; i < offsets[q + 1]; ++i) sim_of[i] = uint16_t(q);
        if (hipMemcpyAsync(c->ws + L.sim_of, sim_of.data(), 2 * n, hipMemcpyHostToDevice, s) != hipSuccess)
            return bail(fail(ABM_E_HIP, "sim index upload failed"));
    }
    launch_pack<T>(b, static_cast<const T*>(pos), static_cast<const T*>(diam), s);
    launch_radius<T>(b, 0, s);
    launch_finish_radius<T>(b, s);
    launch_bbox<T>(b, 0, 0, s);
    if (hipGetLastError() != hipSuccess) return bail(fail(ABM_E_HIP, "init kernels failed to launch"));
    const int rc = read_error(c, true);   // also keeps the host arrays alive until the copies are done
    if (rc != ABM_OK) return bail(rc);
    // The walk: its width, and for the 2-wide walk of one simulation whether
    // the wave shares out its pair terms.  One simulation: from the agents
    // per occupied box of its initial grid (a bitmap of the boxes in the
    // bytes of the per-agent records, free before the first grid build):
    // 4-wide at 4 or more (clustered agents: no uniform packing reaches 3),
    // else 2-wide, shared at 2 or more (several contacts per agent).
    // Otherwise, or when the bitmap does not
    // fit, from the agents per box of the extent: 4-wide at 3 or more (a
    // batch, which always shares), shared at 1.5 or more (about 2 per occupied
    // box where agents spread uniformly).
    c->walk_chunk = p0.walk_chunk;
    c->share = p0.share_terms == 2;
    const bool pick_width = c->walk_chunk == 0, pick_share = p0.share_terms == 0 && nsims == 1;
    bool chosen = false;
    if ((pick_width || pick_share) && nsims == 1) {
        std::vector<int32_t> rep(size_t(kReplicas) * 6);
        if (hipMemcpy(rep.data(), b.bbox_rep, rep.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(ABM_E_HIP, "extent read-back failed"));
        int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (int r = 0; r < kReplicas; ++r)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], rep[size_t(r) * 6 + a]);
                hi[a] = std::max(hi[a], rep[size_t(r) * 6 + 3 + a]);
            }
        uint32_t dims[3] = {0u, 0u, 0u};
        uint64_t nboxes = 1;
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            ok = ok && hi[a] >= lo[a] && int64_t(hi[a]) - int64_t(lo[a]) < (int64_t(1) << 31);
            dims[a] = ok ? uint32_t(int64_t(hi[a]) - int64_t(lo[a]) + 1) : 1u;
            nboxes *= dims[a];
        }
        const uint64_t nwords = (nboxes + 31) / 32;
        if (ok && nboxes < (uint64_t(1) << 40) && 4 * nwords <= uint64_t(16) * uint64_t(cap)) {
            uint32_t* bits = reinterpret_cast<uint32_t*>(c->ws + L.rec);
            unsigned long long* out = reinterpret_cast<unsigned long long*>(c->ws + L.key);
            launch_occupied_boxes<T>(b, lo, dims, bits, nwords, out, s);
            unsigned long long occupied = 0;
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess ||
                hipMemcpy(&occupied, out, 8, hipMemcpyDeviceToHost) != hipSuccess)
                return bail(fail(ABM_E_HIP, "occupied-box count failed"));
            if (occupied > 0) {
                const double per_occupied = double(n) / double(occupied);
                if (pick_width) c->walk_chunk = per_occupied >= 4.0 ? 4 : 2;
                if (pick_share) c->share = per_occupied >= 2.0;
                chosen = true;
            }
        }
    }
    if ((pick_width || pick_share) && !chosen) {
        std::vector<int32_t> rep(size_t(kReplicas) * nsims * 6);
        if (hipMemcpy(rep.data(), b.bbox_rep, rep.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(ABM_E_HIP, "extent read-back failed"));
        double boxes_total = 0.0;
        for (int q = 0; q < nsims; ++q) {
            int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
            for (int r = 0; r < kReplicas; ++r)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], rep[(size_t(r) * nsims + q) * 6 + a]);
                    hi[a] = std::max(hi[a], rep[(size_t(r) * nsims + q) * 6 + 3 + a]);
                }
            double nb = 1.0;
            for (int a = 0; a < 3; ++a) nb *= hi[a] >= lo[a] ? double(hi[a]) - double(lo[a]) + 1.0 : 1.0;
            boxes_total += nb;
        }
        if (pick_width) c->walk_chunk = double(n) >= 3.0 * boxes_total ? 4 : 2;
        if (pick_share) c->share = double(n) >= 1.5 * boxes_total;
    }
    *out = c;
    return ABM_OK;
}

// Zero n bytes at p (a kernel rather than a memset, so that the call records
// no memset node if the caller captures the stream).
__global__ void k_zero_bytes(unsigned char* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

template <class T>
int extent_impl(int64_t n, const void* pos, const void* diam, const abm_params* p, void* scratch, hipStream_t s,
                abm_extent* out, bool zero_by_kernel = false) {
    // scratch: the error word (the only field of Globals the extent kernels
    // touch) in the first 256 bytes, then one SimGrid
    static_assert(offsetof(Globals, err) == 0, "the error word leads Globals");
    static_assert(256 + sizeof(SimGrid) <= ABM_EXTENT_SCRATCH_BYTES, "extent scratch too small");
    char* w = static_cast<char*>(scratch);
    Globals* g = reinterpret_cast<Globals*>(w);
    SimGrid* G = reinterpret_cast<SimGrid*>(w + 256);
    SimGrid h{};
    h.radius = p->interaction_radius;
    h.cell_factor = p->cell_factor;
    if (zero_by_kernel)
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned char*>(w), 256u);
    else
        HIP_TRY(hipMemsetAsync(w, 0, 256, s));
    HIP_TRY(hipMemcpyAsync(G, &h, sizeof(SimGrid), hipMemcpyHostToDevice, s));
    launch_extent<T>(static_cast<const T*>(pos), static_cast<const T*>(diam), uint32_t(n), g, G, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, w, sizeof(err), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&h, G, sizeof(h), hipMemcpyDeviceToHost));
    if (err) return error_code(err);
    out->radius = h.radius;
    out->inv_cell = h.inv_h;
    out->nboxes = 1;
    for (int a = 0; a < 3; ++a) {
        out->cmin[a] = h.bbox[0][a];
        out->dims[a] = int64_t(h.bbox[0][3 + a]) - int64_t(h.bbox[0][a]) + 1;
        out->nboxes *= out->dims[a];
    }
    return ABM_OK;
}

template <class T>
int query_impl(abm_ctx* c, int32_t field, void* dst, int64_t dst_bytes, int32_t dst_is_device) {
    Buffers<T>& b = c->buf<T>();
    const int64_t n = c->n;
    int64_t need = 0;
    int ids_buf = c->ids_cur;
    switch (field) {
        case ABM_FIELD_POSITIONS: need = 3 * n * int64_t(sizeof(T)); break;
        case ABM_FIELD_DIAMETERS: need = n * int64_t(sizeof(T)); break;
        case ABM_FIELD_FORCES:
            if (!c->params.keep_forces) return fail(ABM_E_UNSUPPORTED, "forces are kept only with keep_forces");
            need = 24 * n;
            break;
        case ABM_FIELD_MOVED:
        case ABM_FIELD_STATIC: need = n; break;
        case ABM_FIELD_NNZ: need = 4 * n; break;
        case ABM_FIELD_KEY:
        case ABM_FIELD_PERM:
            if (!c->have_grid) return fail(ABM_E_STATE, "no grid has been built yet (run a step)");
            ids_buf = c->grid_ids;
            need = 4 * n;
            break;
        case ABM_FIELD_STORAGE_IDS: need = 4 * n; break;
        case ABM_FIELD_CELL_START: {
            // box starts are not kept by the step (it counts super-boxes);
            // they are counted here from the boxes of the last grid's agents
            if (!c->have_grid) return fail(ABM_E_STATE, "no grid has been built yet (run a step)");
            if (c->nsims != 1) return fail(ABM_E_UNSUPPORTED, "box starts are kept for a single simulation only");
            HIP_TRY(hipStreamSynchronize(c->stream));
            SimGrid G;
            HIP_TRY(hipMemcpy(&G, b.sims, sizeof(SimGrid), hipMemcpyDeviceToHost));
            if (!G.valid) return fail(ABM_E_GRID, "the last grid is not valid");
            const int64_t nbox = G.nboxes;
            need = 4 * (nbox + 1);
            if (dst_bytes < need) return fail(ABM_E_INVAL, "destination too small: need " + std::to_string(need));
            uint32_t* ranks = reinterpret_cast<uint32_t*>(c->ws + c->L.stage);
            launch_box_ranks<T>(b, c->grid_ids, ranks, c->stream);
            HIP_TRY(hipGetLastError());
            if (const int rc = read_error(c, false)) return rc;
            std::vector<uint32_t> r(n);
            HIP_TRY(hipMemcpy(r.data(), ranks, 4 * n, hipMemcpyDeviceToHost));
            std::vector<uint32_t> start(nbox + 1, 0u);
            for (int64_t k = 0; k < n; ++k) {
                if (r[k] >= uint64_t(nbox)) return fail(ABM_E_HIP, "internal index check failed");
                ++start[r[k] + 1];
            }
            for (int64_t k = 0; k < nbox; ++k) start[k + 1] += start[k];
            HIP_TRY(hipMemcpy(dst, start.data(), need, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
            return ABM_OK;
        }
        case ABM_FIELD_NEIGHBOR_COUNT:
        case ABM_FIELD_NEIGHBORS: {
            if (!c->have_grid) return fail(ABM_E_STATE, "no grid has been built yet (run a step)");
            const bool rowsq = field == ABM_FIELD_NEIGHBORS;
            const int64_t K = rowsq ? dst_bytes / (4 * n) : 0;
            if (rowsq ? K < 1 : dst_bytes < 4 * n)
                return fail(ABM_E_INVAL, "destination too small: need at least " + std::to_string(4 * n) + " bytes");
            if (K > 0xFFFFFFFFll) return fail(ABM_E_INVAL, "row width too large");
            // device target and one word for the largest count, in the staging area when needed
            char* stage = c->ws + c->L.stage;
            uint32_t* worst = reinterpret_cast<uint32_t*>(stage);
            uint32_t* target = static_cast<uint32_t*>(dst);
            if (!dst_is_device) {
                if (4 * n * (rowsq ? K : 1) + 256 > 24 * n)
                    return fail(ABM_E_UNSUPPORTED, "neighbour rows wider than 5 need a device destination");
                target = reinterpret_cast<uint32_t*>(stage + 256);
            }
            HIP_TRY(hipMemsetAsync(worst, 0, 4, c->stream));
            launch_neighbors<T>(b, c->grid_ids, rowsq ? nullptr : target, rowsq ? target : nullptr, uint32_t(K), worst,
                                c->stream);
            HIP_TRY(hipGetLastError());
            uint32_t w = 0;
            HIP_TRY(hipMemcpyAsync(&w, worst, 4, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            if (const int rc = read_error(c, false)) return rc;
            if (rowsq && w > K)
                return fail(ABM_E_INVAL, "row width " + std::to_string(K) + " too small: need " + std::to_string(w));
            if (!dst_is_device)
                HIP_TRY(hipMemcpy(dst, target, 4 * n * (rowsq ? K : 1), hipMemcpyDeviceToHost));
            return ABM_OK;
        }
        case ABM_FIELD_EXTENT: {
            need = 56 * int64_t(c->nsims);
            if (dst_bytes < need) return fail(ABM_E_INVAL, "destination too small: need " + std::to_string(need));
            HIP_TRY(hipStreamSynchronize(c->stream));
            std::vector<SimGrid> sims(c->nsims);
            HIP_TRY(hipMemcpy(sims.data(), b.sims, sizeof(SimGrid) * c->nsims, hipMemcpyDeviceToHost));
            std::vector<int64_t> v(7 * c->nsims);
            for (int s = 0; s < c->nsims; ++s) {
                for (int a = 0; a < 3; ++a) {
                    v[7 * s + a] = sims[s].cmin[a];
                    v[7 * s + 3 + a] = sims[s].dims[a];
                }
                v[7 * s + 6] = sims[s].nboxes;
            }
            HIP_TRY(hipMemcpy(dst, v.data(), need, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
            return ABM_OK;
        }
        default: return fail(ABM_E_INVAL, "unknown field");
    }
    if (dst_bytes < need) return fail(ABM_E_INVAL, "destination too small: need " + std::to_string(need));
    void* target = dst_is_device ? dst : static_cast<void*>(c->ws + c->L.stage);
    if (field == ABM_FIELD_POSITIONS)
        launch_unpack_positions<T>(b, c->pos_cur, ids_buf, static_cast<T*>(target), c->stream);
    else if (field == ABM_FIELD_KEY)
        launch_box_ranks<T>(b, ids_buf, static_cast<uint32_t*>(target), c->stream);
    else if (field == ABM_FIELD_PERM)
        launch_canonical_ids<T>(b, ids_buf, last_grid_starts<T>(c), static_cast<uint32_t*>(target), c->stream);
    else
        launch_unpack_field<T>(b, c->pos_cur, ids_buf, field, target, c->stream);
    HIP_TRY(hipGetLastError());
    const int rc = read_error(c, false);
    if (rc != ABM_OK) return rc;
    if (!dst_is_device) HIP_TRY(hipMemcpy(dst, target, need, hipMemcpyDeviceToHost));
    return ABM_OK;
}

struct StateHeader {
    uint64_t magic;
    int64_t n;
    int64_t step;
    int32_t precision;
    int32_t nsims;
};
constexpr uint64_t kStateMagic = 0x3165746174534241ull;  // "ABState1" in little-endian bytes

int64_t state_bytes(abm_ctx* c) { return int64_t(sizeof(StateHeader)) + c->n * (3 * c->elem() + 1 + 4); }

template <class T>
int import_impl(abm_ctx* c, const void* src, int64_t src_bytes) {
    if (src_bytes < state_bytes(c)) return fail(ABM_E_INVAL, "state buffer too small");
    StateHeader h;
    std::memcpy(&h, src, sizeof(h));
    if (h.magic != kStateMagic || h.n != c->n || h.precision != c->precision || h.nsims != c->nsims)
        return fail(ABM_E_INVAL, "state does not match this context");
    Buffers<T>& b = c->buf<T>();
    const char* p = static_cast<const char*>(src) + sizeof(h);
    char* stage = c->ws + c->L.stage;
    const int64_t pos_b = 3 * c->n * int64_t(sizeof(T));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(stage, p, pos_b, hipMemcpyHostToDevice));
    launch_load_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<const T*>(stage), c->stream);
    c->inc_ready = false;   // positions replaced outside the step
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(stage, p + pos_b, c->n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(stage + align_up(c->n), p + pos_b + c->n, 4 * c->n, hipMemcpyHostToDevice));
    launch_set_flags<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<const uint8_t*>(stage),
                        reinterpret_cast<const int32_t*>(stage + align_up(c->n)), c->stream);
    c->step = h.step;
    enqueue_extent<T>(c);
    HIP_TRY(hipGetLastError());
    return read_error(c, true);
}

template <class T>
int export_impl(abm_ctx* c, void* dst, int64_t dst_bytes) {
    if (dst_bytes < state_bytes(c)) return fail(ABM_E_INVAL, "destination too small");
    StateHeader h{kStateMagic, c->n, c->step, c->precision, c->nsims};
    std::memcpy(dst, &h, sizeof(h));
    char* p = static_cast<char*>(dst) + sizeof(h);
    const int64_t pos_b = 3 * c->n * int64_t(sizeof(T));
    int rc = query_impl<T>(c, ABM_FIELD_POSITIONS, p, pos_b, 0);
    if (rc == ABM_OK) rc = query_impl<T>(c, ABM_FIELD_MOVED, p + pos_b, c->n, 0);
    if (rc == ABM_OK) rc = query_impl<T>(c, ABM_FIELD_NNZ, p + pos_b + c->n, 4 * c->n, 0);
    return rc;
}

// ---------------------------------------------------------------- adjoint
// The record: checkpoints, one segment's positions, x_T, lambda twice and w,
// then (optional) a word per taped step and the contact tapes, one per step.
struct RecLayout {
    int64_t ckpt, seg, xT, lam, lam2, w, total;   // total: without tapes
    int64_t worst, tape, tape_step;               // the tapes: first one, bytes of each
    int64_t total_seg, total_all;                 // with one segment's tapes, with every step's
    int32_t nckpt;
};

RecLayout rec_layout(abm_ctx* c, int32_t nsteps, int32_t ckpt_every) {
    RecLayout r{};
    const int64_t pb = align_up(3 * c->n * c->elem());
    const int64_t db = align_up(24 * c->n);
    r.nckpt = (nsteps + ckpt_every - 1) / ckpt_every;
    int64_t off = 0;
    r.ckpt = off;
    off += pb * r.nckpt;
    r.seg = off;
    off += pb * ckpt_every;
    r.xT = off;
    off += pb;
    r.lam = off;
    off += db;
    r.lam2 = off;
    off += db;
    r.w = off;
    off += db;
    r.total = off;
    r.worst = off;
    off += align_up(4 * int64_t(nsteps));
    r.tape = off;
    r.tape_step = align_up(4 * c->n * c->elem()) + 2 * align_up(4 * c->n) + align_up(4 * c->n * kTapeWidth);
    r.total_seg = off + r.tape_step * std::min(ckpt_every, nsteps);
    r.total_all = off + r.tape_step * nsteps;
    return r;
}

TapeStep tape_at(abm_ctx* c, const RecLayout& R, char* base, int32_t k) {
    char* p = base + R.tape + R.tape_step * k;
    TapeStep tp;
    tp.pos = p;
    p += align_up(4 * c->n * c->elem());
    tp.ids = reinterpret_cast<uint32_t*>(p);
    p += align_up(4 * c->n);
    tp.cnt = reinterpret_cast<uint32_t*>(p);
    p += align_up(4 * c->n);
    tp.list = reinterpret_cast<uint32_t*>(p);
    tp.worst = reinterpret_cast<uint32_t*>(base + R.worst) + k;
    return tp;
}

// The largest contact counts of taped steps [0, m), read back to the host.
int read_worst(abm_ctx* c, const RecLayout& R, char* base, int32_t m, std::vector<uint32_t>& out) {
    out.assign(size_t(m), 0u);
    HIP_TRY(hipMemcpyAsync(out.data(), base + R.worst, 4 * size_t(m), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (uint32_t v : out) c->rec_worst = std::max(c->rec_worst, v);
    return ABM_OK;
}

template <class T>
int forward_record_impl(abm_ctx* c, int32_t nsteps, int32_t ckpt_every, void* rec, int64_t rec_bytes) {
    const RecLayout R = rec_layout(c, nsteps, ckpt_every);
    if (rec_bytes < R.total) return fail(ABM_E_WORKSPACE, "record buffer too small: need " + std::to_string(R.total));
    Buffers<T>& b = c->buf<T>();
    char* base = static_cast<char*>(rec);
    const int64_t pb = align_up(3 * c->n * c->elem());
    const int tapes = rec_bytes >= R.total_all ? 2 : (rec_bytes >= R.total_seg ? 1 : 0);
    c->recorded = false;
    c->rec_start = c->step;
    c->rec_worst = 0;
    if (tapes == 2) HIP_TRY(hipMemsetAsync(base + R.worst, 0, 4 * size_t(nsteps), c->stream));
    for (int32_t s = 0; s < nsteps; ++s) {
        if (s % ckpt_every == 0)
            launch_unpack_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<T*>(base + R.ckpt + pb * (s / ckpt_every)),
                                       c->stream);
        if (tapes == 2) {
            c->tape_next = tape_at(c, R, base, s);
            c->inc_ready = false;   // a taped step's grid is a full build
        }
        int rc = do_steps<T>(c, 1, true);
        if (rc != ABM_OK) return rc;
    }
    launch_unpack_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<T*>(base + R.xT), c->stream);
    HIP_TRY(hipGetLastError());
    int rc = read_error(c, true);
    if (rc != ABM_OK) return rc;
    c->rec_tapes = tapes;
    if (tapes == 2) {
        std::vector<uint32_t> worst;
        if ((rc = read_worst(c, R, base, nsteps, worst)) != ABM_OK) return rc;
        // an incomplete tape: the backward recomputes each segment, taping
        // the steps again and walking the grid of those that do not fit
        if (c->rec_worst > kTapeWidth) c->rec_tapes = 1;
    }
    c->recorded = true;
    c->rec_steps = nsteps;
    c->rec_ckpt = ckpt_every;
    c->rec = base;
    c->rec_bytes = rec_bytes;
    return ABM_OK;
}

// The grid of the current positions and its tape, without the step's force
// (the last step of a recomputed segment: its new positions are not needed).
template <class T>
void enqueue_tape_only(abm_ctx* c, const TapeStep& tp) {
    Buffers<T>& b = c->buf<T>();
    c->inc_ready = false;   // a taped step's grid is a full build
    guard_stamps<T>(c, 1);
    set_grid_pos<T>(c, c->pos_cur);
    launch_setup<T>(b, int(c->step & 1), c->inc_ready, c->stream);
    launch_grid<T>(b, c->pos_cur, c->ids_cur, false, false, c->stream);
    swap_cell_start<T>(c);
    launch_adj_tape<T>(b, c->ids_cur, tp, c->stream);
    c->grid_ids = c->ids_cur;
    c->inc_ready = false;
    c->stamp_count += 1;
}

// Load positions (by id) into the current storage and build the grid for them.
template <class T>
void load_and_grid(abm_ctx* c, const T* pos_by_id) {
    Buffers<T>& b = c->buf<T>();
    launch_load_positions<T>(b, c->pos_cur, c->ids_cur, pos_by_id, c->stream);
    c->inc_ready = false;   // positions replaced outside the step
    launch_bbox<T>(b, c->pos_cur, 0, c->stream);
    guard_stamps<T>(c, 1);
    set_grid_pos<T>(c, c->pos_cur);
    launch_setup<T>(b, 0, false, c->stream);
    launch_grid<T>(b, c->pos_cur, c->ids_cur, false, false, c->stream);
    swap_cell_start<T>(c);
    c->grid_ids = c->ids_cur;
    c->inc_ready = false;
    c->stamp_count += 1;
}

template <class T>
int backward_impl(abm_ctx* c, const double* dL_dxT, double* dL_dx0, double* dL_dparams) {
    if (!c->recorded) return fail(ABM_E_STATE, "abm_backward needs a preceding abm_forward_record");
    Buffers<T>& b = c->buf<T>();
    const RecLayout R = rec_layout(c, c->rec_steps, c->rec_ckpt);
    char* base = c->rec;
    const int64_t pb = align_up(3 * c->n * c->elem());
    double* lam = reinterpret_cast<double*>(base + R.lam);
    double* lam2 = reinterpret_cast<double*>(base + R.lam2);
    double* w = reinterpret_cast<double*>(base + R.w);
    const uint32_t n = uint32_t(c->n);
    hipStream_t s = c->stream;
    const int64_t end_step = c->step;
    // lambda is kept by id, as dL/dx_T and dL/dx_0 are
    HIP_TRY(hipMemcpyAsync(lam, dL_dxT, 24 * size_t(n), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(dL_dparams, 0, 2 * sizeof(double), s));
    const int nblocks = adj_blocks(n);
    c->taped_reverse = 0;
    // one reverse step on the tape of step t, or on a grid built from x_t
    auto reverse_taped = [&](const TapeStep& tp) {
        launch_adj_tape_w<T>(b, tp, lam, w, s);
        launch_adj_tape_gather<T>(b, tp, lam, w, lam2, s);
        launch_adj_finish<T>(b, nblocks, dL_dparams, s);
        std::swap(lam, lam2);
        c->taped_reverse += 1;
    };
    auto reverse_walked = [&](const T* x_t) {
        load_and_grid<T>(c, x_t);
        launch_adj_w<T>(b, c->ids_cur, lam, w, s);
        launch_adj_gather<T>(b, c->ids_cur, lam, w, lam2, s);
        launch_adj_finish<T>(b, nblocks, dL_dparams, s);
        std::swap(lam, lam2);
    };
    if (c->rec_tapes == 2) {
        for (int32_t t = c->rec_steps - 1; t >= 0; --t) reverse_taped(tape_at(c, R, base, t));
    } else {
        std::vector<uint32_t> worst;
        for (int32_t seg = R.nckpt - 1; seg >= 0; --seg) {
            const int32_t s0 = seg * c->rec_ckpt;
            const int32_t s1 = std::min(c->rec_steps, s0 + c->rec_ckpt);
            const bool taped = c->rec_tapes == 1;
            // recompute the segment forward, keeping every step's positions
            // (and contacts); the step out of its last state is not needed
            launch_load_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<const T*>(base + R.ckpt + pb * seg), s);
            c->inc_ready = false;   // positions replaced outside the step
            launch_mark_moved<T>(b, c->pos_cur, s);
            c->step = c->rec_start + s0;
            enqueue_extent<T>(c);
            if (taped) HIP_TRY(hipMemsetAsync(base + R.worst, 0, 4 * size_t(s1 - s0), s));
            for (int32_t t = s0; t < s1; ++t) {
                launch_unpack_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<T*>(base + R.seg + pb * (t - s0)), s);
                if (t + 1 < s1) {
                    if (taped) {
                        c->tape_next = tape_at(c, R, base, t - s0);
                        c->inc_ready = false;   // a taped step's grid is a full build
                    }
                    int rc = do_steps<T>(c, 1, true);
                    if (rc != ABM_OK) return rc;
                } else if (taped) {
                    enqueue_tape_only<T>(c, tape_at(c, R, base, t - s0));
                }
            }
            if (taped) {
                HIP_TRY(hipGetLastError());
                if (int rc = read_worst(c, R, base, s1 - s0, worst)) return rc;
            }
            // walk the segment backward
            for (int32_t t = s1 - 1; t >= s0; --t) {
                if (taped && worst[size_t(t - s0)] <= kTapeWidth)
                    reverse_taped(tape_at(c, R, base, t - s0));
                else
                    reverse_walked(reinterpret_cast<const T*>(base + R.seg + pb * (t - s0)));
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(dL_dx0, lam, 24 * size_t(n), hipMemcpyDeviceToDevice, s));
    // restore the final state of the recorded run
    launch_load_positions<T>(b, c->pos_cur, c->ids_cur, reinterpret_cast<const T*>(base + R.xT), s);
    c->inc_ready = false;   // positions replaced outside the step
    c->step = end_step;
    enqueue_extent<T>(c);
    HIP_TRY(hipGetLastError());
    return read_error(c, true);
}

template <class T>
int graph_capture_impl(abm_ctx* c, int32_t nsteps) {
    const int se = c->params.sort_every;
    if (nsteps % 2 != 0 || (se > 0 && nsteps % se != 0))
        return fail(ABM_E_INVAL, "graph steps must be even and a multiple of sort_every, so replays start from the same buffers");
    int32_t relayouts = 0;
    for (int32_t t = 0; t < nsteps; ++t)
        if (se > 0 && ((c->step + t + 1) % se == 0)) ++relayouts;
    if (relayouts % 2 != 0)
        return fail(ABM_E_INVAL, "graph must contain an even number of re-layout steps");
    if (nsteps > int32_t(kStampPeriod)) return fail(ABM_E_INVAL, "at most 32767 steps per graph");
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    // make sure no stamp wrap can fall inside a replay: replays start from a cleared table
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int64_t saved_step = c->step;
    const int saved_pos = c->pos_cur, saved_ids = c->ids_cur;
    const uint32_t saved_stamp = c->stamp_count;
    const bool saved_inc = c->inc_ready;
    const int saved_grid_pos = c->grid_pos;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    launch_clear_cellinfo<T>(c->buf<T>(), c->stream);
    c->stamp_count = 0;
    c->inc_ready = false;   // a replay starts from a cleared table: its first grid is a full build
    for (int32_t t = 0; t < nsteps; ++t) enqueue_step<T>(c, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->graph_grid_ids = c->grid_ids;
    c->graph_inc_after = c->inc_ready;
    c->step = saved_step;
    c->pos_cur = saved_pos;
    c->ids_cur = saved_ids;
    c->stamp_count = saved_stamp;
    c->inc_ready = saved_inc;   // the captured steps did not run (cell_start parity is back: even steps)
    set_grid_pos<T>(c, saved_grid_pos);
    if (e != hipSuccess) return fail(ABM_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    c->graph = g;
    HIP_TRY(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    c->graph_steps = nsteps;
    return ABM_OK;
}

template <class T>
int graph_launch_impl(abm_ctx* c) {
    if (!c->graph_exec) return fail(ABM_E_STATE, "no graph captured");
    HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
    // a replay advances the state exactly as the captured steps do; buffer
    // indices return to their start because the step counts are even
    c->step += c->graph_steps;
    c->stamp_count = uint32_t(c->graph_steps);
    c->grid_ids = c->graph_grid_ids;
    c->inc_ready = c->graph_inc_after;
    c->have_grid = true;
    // the last captured step built its grid in the copy the state left
    // (an even number of steps returns the state to where it started)
    set_grid_pos<T>(c, c->pos_cur ^ 1);
    return ABM_OK;
}

template <class T>
int dispatch_steps(abm_ctx* c, int32_t nsteps) { return do_steps<T>(c, nsteps, true); }

// ---------------------------------------------------------------- population
// After agents were added or removed: the new population's extent for the
// next step, whose grid is a full build; the last grid, a captured graph and
// a recorded forward run no longer apply.
template <class T>
int population_changed(abm_ctx* c, int64_t n) {
    c->n = n;
    c->offsets.back() = n;
    Buffers<T>& b = c->buf<T>();
    b.n = uint32_t(n);
    launch_set_population(b.sims, uint32_t(n), c->stream);
    c->inc_ready = false;
    c->have_grid = false;
    c->recorded = false;
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    enqueue_extent<T>(c);
    HIP_TRY(hipGetLastError());
    return read_error(c, true);
}

template <class T>
int add_impl(abm_ctx* c, int64_t m, const void* pos, const void* diam) {
    if (c->nsims != 1) return fail(ABM_E_UNSUPPORTED, "agents are added to single-simulation contexts only");
    if (m < 0 || (m > 0 && (!pos || !diam))) return fail(ABM_E_INVAL, "bad arguments");
    if (c->n + m > c->cap)
        return fail(ABM_E_INVAL, "capacity exceeded: " + std::to_string(c->n + m) + " > " + std::to_string(c->cap));
    if (m == 0) return ABM_OK;
    if (const int rc = read_error(c, true)) return rc;
    Buffers<T>& b = c->buf<T>();
    launch_add<T>(b, c->pos_cur, c->ids_cur, uint32_t(c->n), uint32_t(m), static_cast<const T*>(pos),
                  static_cast<const T*>(diam), c->stream);
    HIP_TRY(hipGetLastError());
    // the new agents went to slots past the population, where the last
    // grid's append region lies: that grid cannot be queried any more.  A
    // rejected agent leaves the population as it was.
    c->have_grid = false;
    if (const int rc = read_error(c, true)) return rc;
    return population_changed<T>(c, c->n + m);
}

template <class T>
int remove_impl(abm_ctx* c, int64_t m, const int64_t* ids) {
    if (c->nsims != 1) return fail(ABM_E_UNSUPPORTED, "agents are removed from single-simulation contexts only");
    if (m < 0 || m > c->n || (m > 0 && !ids)) return fail(ABM_E_INVAL, "bad arguments");
    if (m == 0) return ABM_OK;
    if (m == c->n) return fail(ABM_E_INVAL, "a context keeps at least one agent");
    if (const int rc = read_error(c, true)) return rc;
    Buffers<T>& b = c->buf<T>();
    uint32_t* work = reinterpret_cast<uint32_t*>(c->ws + c->L.stage);
    launch_remove<T>(b, c->pos_cur, c->ids_cur, uint32_t(m), ids, work, uint32_t(c->cap), c->stream, 0);
    HIP_TRY(hipGetLastError());
    // bad or repeated ids are reported before anything moves
    if (const int rc = read_error(c, true)) return rc;
    launch_remove<T>(b, c->pos_cur, c->ids_cur, uint32_t(m), ids, work, uint32_t(c->cap), c->stream, 1);
    HIP_TRY(hipGetLastError());
    c->pos_cur ^= 1;
    c->ids_cur ^= 1;
    return population_changed<T>(c, c->n - m);
}

template <class T>
int diameters_impl(abm_ctx* c, int64_t m, const int64_t* ids, const void* diam) {
    if (m < 0 || m > c->n || (m > 0 && (!ids || !diam))) return fail(ABM_E_INVAL, "bad arguments");
    if (m == 0) return ABM_OK;
    if (const int rc = read_error(c, true)) return rc;
    Buffers<T>& b = c->buf<T>();
    uint32_t* mk = reinterpret_cast<uint32_t*>(c->ws + c->L.stage);
    const T* d = static_cast<const T*>(diam);
    launch_set_diameters<T>(b, c->pos_cur, c->ids_cur, uint32_t(m), ids, d, mk, c->stream, 0);
    HIP_TRY(hipGetLastError());
    // bad ids or diameters are reported before anything changes
    if (const int rc = read_error(c, true)) return rc;
    launch_set_diameters<T>(b, c->pos_cur, c->ids_cur, uint32_t(m), ids, d, mk, c->stream, 1);
    HIP_TRY(hipGetLastError());
    // positions, boxes and the population are as they were, so the last grid,
    // the next step's update build and a captured graph still apply; a
    // recorded forward run used the old diameters
    c->recorded = false;
    return read_error(c, true);
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

int abm_abi_version(void) { return ABM_ABI_VERSION; }

void abm_default_params(abm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->k = 2.0;
    p->gamma = 1.0;
    p->mu = 0.1;
    p->f_adh = 0.0;
    p->delta_max = 3.0;
    p->interaction_radius = 0.0;
    p->cell_factor = 1.0;
    p->precision = ABM_F32;
    p->detect_static = 0;
    p->sort_every = 1;
    p->block_size = 256;
    p->keep_forces = 0;
    p->walk_chunk = 0;
    p->super_fraction = 0.0;
}

const char* abm_last_error(void) { return g_last_error.c_str(); }

int abm_extent_of(int64_t n, const void* pos, const void* diam, const abm_params* p, void* scratch, void* stream,
                  abm_extent* out) {
    std::string why;
    if (!valid_params(p, &why)) return fail(ABM_E_INVAL, why);
    if (n <= 0 || n > 0xFFFFFFFEll || !pos || !diam || !scratch || !out) return fail(ABM_E_INVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(scratch) % 8) return fail(ABM_E_INVAL, "scratch must be 8-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return p->precision == ABM_F64 ? extent_impl<double>(n, pos, diam, p, scratch, s, out)
                                   : extent_impl<float>(n, pos, diam, p, scratch, s, out);
}

}  // extern "C"

// ------------------------------------------------ extent without allocation
// The scratch of abm_extent_of_noalloc: the error word and one SimGrid, as
// abm_extent_of's caller-owned scratch holds them.  Each GPU the library runs
// on holds its own copy until the process ends; host code never passes the
// array's name to a kernel or a copy, only the device address
// hipGetSymbolAddress gives for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[ABM_EXTENT_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch, looked up on the first call
// on that device.
int device_scratch(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(ABM_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ABM_E_HIP, "hipGetSymbolAddress gave a null address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ABM_OK;
}
}  // namespace

extern "C" {

int abm_extent_of_noalloc(int64_t n, const void* pos, const void* diam, const abm_params* p, void* stream,
                          abm_extent* out) {
    std::string why;
    if (!valid_params(p, &why)) return fail(ABM_E_INVAL, why);
    if (n <= 0 || n > ABM_NOALLOC_MAX_AGENTS)
        return fail(ABM_E_INVAL, "n must be in [1, ABM_NOALLOC_MAX_AGENTS = 2^32 - 2]");
    if (!pos || !diam || !out) return fail(ABM_E_INVAL, "bad arguments");
    void* ptr = nullptr;
    if (int rc = device_scratch(&ptr)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return p->precision == ABM_F64 ? extent_impl<double>(n, pos, diam, p, ptr, s, out, true)
                                   : extent_impl<float>(n, pos, diam, p, ptr, s, out, true);
}

int abm_workspace_bytes(int32_t nsims, const int64_t* offsets, const int64_t* box_capacity, const abm_params* p,
                        int64_t* bytes) {
    std::string why;
    if (!valid_params(p, &why)) return fail(ABM_E_INVAL, why);
    if (nsims < 1 || nsims > 65535 || !offsets || !box_capacity || !bytes) return fail(ABM_E_INVAL, "bad arguments");
    const int64_t n = offsets[nsims];
    if (offsets[0] != 0 || n <= 0 || n > kMaxAgents)
        return fail(ABM_E_INVAL, "offsets must start at 0, n in [1, 2^31 - 2^20]");
    int64_t boxes = 0, supers = 0;
    for (int s = 0; s < nsims; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(ABM_E_INVAL, "offsets must be non-decreasing");
        if (box_capacity[s] < 1) return fail(ABM_E_INVAL, "box capacity must be >= 1");
        boxes += box_capacity[s];
        supers += super_capacity(box_capacity[s], p->super_fraction);
    }
    if (boxes >= 0xFFFFFFFFll) return fail(ABM_E_GRID, "total box capacity must be below 2^32");
    *bytes = make_layout(n, nsims, supers, p->keep_forces != 0, p->precision == ABM_F64 ? 8 : 4).total;
    return ABM_OK;
}

int abm_init(abm_ctx** ctx, int64_t n, const void* pos, const void* diam, const abm_params* p, int64_t box_capacity,
             void* ws, int64_t ws_bytes, void* stream) {
    if (!ctx || !pos || !diam || !p || n <= 0 || n > 0xFFFFFFFEll) return fail(ABM_E_INVAL, "bad arguments");
    const int64_t offsets[2] = {0, n};
    return p->precision == ABM_F64
               ? init_impl<double>(ctx, 1, offsets, pos, diam, p, &box_capacity, ws, ws_bytes, stream, 0)
               : init_impl<float>(ctx, 1, offsets, pos, diam, p, &box_capacity, ws, ws_bytes, stream, 0);
}

int abm_workspace_bytes_capacity(int64_t capacity, int64_t box_capacity, const abm_params* p, int64_t* bytes) {
    std::string why;
    if (!p || !valid_params(p, &why)) return fail(ABM_E_INVAL, p ? why : "params is null");
    if (!bytes || capacity < 1 || capacity > kMaxAgents) return fail(ABM_E_INVAL, "capacity must be in [1, 2^31 - 2^20]");
    if (box_capacity < 1 || box_capacity >= 0xFFFFFFFFll) return fail(ABM_E_INVAL, "box capacity must be in [1, 2^32 - 1)");
    *bytes = make_layout(capacity, 1, super_capacity(box_capacity, p->super_fraction), p->keep_forces != 0,
                         p->precision == ABM_F64 ? 8 : 4).total;
    return ABM_OK;
}

int abm_init_capacity(abm_ctx** ctx, int64_t n, int64_t capacity, const void* pos, const void* diam,
                      const abm_params* p, int64_t box_capacity, void* ws, int64_t ws_bytes, void* stream) {
    if (!ctx || !pos || !diam || !p || n <= 0 || capacity < n) return fail(ABM_E_INVAL, "bad arguments");
    const int64_t offsets[2] = {0, n};
    return p->precision == ABM_F64
               ? init_impl<double>(ctx, 1, offsets, pos, diam, p, &box_capacity, ws, ws_bytes, stream, capacity)
               : init_impl<float>(ctx, 1, offsets, pos, diam, p, &box_capacity, ws, ws_bytes, stream, capacity);
}

int abm_add_agents(abm_ctx* c, int64_t m, const void* pos, const void* diam) {
    if (int rc = check_ctx(c)) return rc;
    return c->precision == ABM_F64 ? add_impl<double>(c, m, pos, diam) : add_impl<float>(c, m, pos, diam);
}

int abm_remove_agents(abm_ctx* c, int64_t m, const int64_t* ids) {
    if (int rc = check_ctx(c)) return rc;
    return c->precision == ABM_F64 ? remove_impl<double>(c, m, ids) : remove_impl<float>(c, m, ids);
}

int abm_set_diameters(abm_ctx* c, int64_t m, const int64_t* ids, const void* diam) {
    if (int rc = check_ctx(c)) return rc;
    return c->precision == ABM_F64 ? diameters_impl<double>(c, m, ids, diam) : diameters_impl<float>(c, m, ids, diam);
}

int abm_population(abm_ctx* c, int64_t* n, int64_t* capacity) {
    if (int rc = check_ctx(c)) return rc;
    if (n) *n = c->n;
    if (capacity) *capacity = c->cap;
    return ABM_OK;
}

int abm_init_batched(abm_ctx** ctx, int32_t nsims, const int64_t* offsets, const void* pos, const void* diam,
                     const abm_params* per_sim, const int64_t* box_capacity, void* ws, int64_t ws_bytes,
                     void* stream) {
    if (!ctx || nsims < 1 || nsims > 65535 || !offsets || !pos || !diam || !per_sim || !box_capacity)
        return fail(ABM_E_INVAL, "bad arguments");
    if (offsets[0] != 0 || offsets[nsims] > 0xFFFFFFFEll) return fail(ABM_E_INVAL, "bad offsets");
    for (int s = 0; s < nsims; ++s)
        if (per_sim[s].precision != per_sim[0].precision) return fail(ABM_E_INVAL, "all simulations need one precision");
    return per_sim[0].precision == ABM_F64
               ? init_impl<double>(ctx, nsims, offsets, pos, diam, per_sim, box_capacity, ws, ws_bytes, stream, 0)
               : init_impl<float>(ctx, nsims, offsets, pos, diam, per_sim, box_capacity, ws, ws_bytes, stream, 0);
}

int abm_set_params(abm_ctx* c, const abm_params* p) {
    if (int rc = check_ctx(c)) return rc;
    std::string why;
    if (!valid_params(p, &why)) return fail(ABM_E_INVAL, why);
    if (p->precision != c->precision) return fail(ABM_E_INVAL, "precision cannot change");
    if (p->keep_forces && c->L.force[0] < 0) return fail(ABM_E_UNSUPPORTED, "workspace has no force buffers");
    if (p->cell_factor != c->params.cell_factor || p->interaction_radius != c->params.interaction_radius ||
        p->order != c->params.order)
        return fail(ABM_E_UNSUPPORTED, "the grid geometry is fixed at init");
    const bool force_law_changed = p->k != c->params.k || p->gamma != c->params.gamma || p->mu != c->params.mu ||
                                   p->f_adh != c->params.f_adh || p->delta_max != c->params.delta_max;
    launch_set_params(c->precision == ABM_F64 ? c->bd.sims : c->bf.sims, c->nsims, p->k, p->gamma, p->mu, p->f_adh,
                      p->delta_max, c->stream);
    if (force_law_changed) {
        if (c->precision == ABM_F64)
            launch_mark_moved<double>(c->bd, c->pos_cur, c->stream);
        else
            launch_mark_moved<float>(c->bf, c->pos_cur, c->stream);
    }
    const int keep = p->keep_forces;
    c->params.k = p->k;
    c->params.gamma = p->gamma;
    c->params.mu = p->mu;
    c->params.f_adh = p->f_adh;
    c->params.delta_max = p->delta_max;
    c->params.detect_static = p->detect_static;
    c->params.sort_every = p->sort_every;
    c->params.block_size = p->block_size;
    c->params.keep_forces = keep;
    if (p->walk_chunk) c->walk_chunk = p->walk_chunk;
    c->params.walk_chunk = p->walk_chunk;
    if (p->share_terms) c->share = p->share_terms == 2;
    c->params.share_terms = p->share_terms;
    HIP_TRY(hipGetLastError());
    return ABM_OK;
}

int abm_step(abm_ctx* c, int32_t nsteps) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps < 0) return fail(ABM_E_INVAL, "nsteps must be >= 0");
    c->recorded = false;
    return c->precision == ABM_F64 ? dispatch_steps<double>(c, nsteps) : dispatch_steps<float>(c, nsteps);
}

int abm_sync(abm_ctx* c) {
    if (int rc = check_ctx(c)) return rc;
    return read_error(c, true);
}

int abm_query(abm_ctx* c, int32_t field, void* dst, int64_t dst_bytes, int32_t dst_is_device) {
    if (int rc = check_ctx(c)) return rc;
    if (!dst) return fail(ABM_E_INVAL, "null destination");
    return c->precision == ABM_F64 ? query_impl<double>(c, field, dst, dst_bytes, dst_is_device)
                                   : query_impl<float>(c, field, dst, dst_bytes, dst_is_device);
}

int abm_get_stats(abm_ctx* c, abm_stats* out) {
    if (int rc = check_ctx(c)) return rc;
    if (!out) return fail(ABM_E_INVAL, "null output");
    HIP_TRY(hipStreamSynchronize(c->stream));
    Globals g{};
    HIP_TRY(hipMemcpy(&g, c->ws + c->L.globals, sizeof(g), hipMemcpyDeviceToHost));
    out->step = c->step;
    const int last = int((c->step - 1) & 1);
    int64_t ns = 0, nm = 0;
    double fs[3] = {0.0, 0.0, 0.0};
    uint64_t dm = 0;
    for (int r = 0; r < kReplicas; ++r) {   // replicas in order
        ns += int64_t(g.stats[last][r][0]);
        nm += int64_t(g.stats[last][r][1]);
        for (int a = 0; a < 3; ++a) fs[a] += g.fsum[last][r][a];
        dm = std::max<uint64_t>(dm, g.dmax[last][r]);
    }
    const bool any = c->step > 0;
    out->n_static = any ? ns : 0;
    out->n_moved = any ? nm : 0;
    out->error = g.err;
    out->build = (g.inc ? 1u : 0u) | (g.rebuilt << 1);
    double dmax = 0.0;
    std::memcpy(&dmax, &dm, sizeof(dmax));
    for (int a = 0; a < 3; ++a) out->sum_force[a] = any ? fs[a] : 0.0;
    out->max_displacement = any ? dmax : 0.0;
    out->skip_fraction = any && c->n > 0 ? double(ns) / double(c->n) : 0.0;
    return ABM_OK;
}

int abm_state_bytes(abm_ctx* c, int64_t* bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (!bytes) return fail(ABM_E_INVAL, "null output");
    *bytes = state_bytes(c);
    return ABM_OK;
}

int abm_export_state(abm_ctx* c, void* dst, int64_t dst_bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (!dst) return fail(ABM_E_INVAL, "null destination");
    return c->precision == ABM_F64 ? export_impl<double>(c, dst, dst_bytes) : export_impl<float>(c, dst, dst_bytes);
}

int abm_import_state(abm_ctx* c, const void* src, int64_t src_bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (!src) return fail(ABM_E_INVAL, "null source");
    c->recorded = false;
    return c->precision == ABM_F64 ? import_impl<double>(c, src, src_bytes) : import_impl<float>(c, src, src_bytes);
}

int abm_graph_capture(abm_ctx* c, int32_t nsteps) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps <= 0) return fail(ABM_E_INVAL, "nsteps must be > 0");
    if (!c->stream) return fail(ABM_E_INVAL, "graph capture needs a stream other than the null stream");
    return c->precision == ABM_F64 ? graph_capture_impl<double>(c, nsteps) : graph_capture_impl<float>(c, nsteps);
}

int abm_graph_launch(abm_ctx* c) {
    if (int rc = check_ctx(c)) return rc;
    c->recorded = false;
    return c->precision == ABM_F64 ? graph_launch_impl<double>(c) : graph_launch_impl<float>(c);
}

// a record of every step's tapes must stay far below 2^63 bytes
static bool record_fits(abm_ctx* c, int32_t nsteps) {
    return double(rec_layout(c, 1, 1).tape_step + 4 * c->n * c->elem()) * double(nsteps) < 1e18;
}

int abm_record_bytes(abm_ctx* c, int32_t nsteps, int32_t ckpt_every, int64_t* bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps < 1 || ckpt_every < 1 || !bytes) return fail(ABM_E_INVAL, "bad arguments");
    if (!record_fits(c, nsteps)) return fail(ABM_E_INVAL, "record too large");
    *bytes = rec_layout(c, nsteps, ckpt_every).total_all;
    return ABM_OK;
}

int abm_record_sizes(abm_ctx* c, int32_t nsteps, int32_t ckpt_every, int64_t* sizes) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps < 1 || ckpt_every < 1 || !sizes) return fail(ABM_E_INVAL, "bad arguments");
    if (!record_fits(c, nsteps)) return fail(ABM_E_INVAL, "record too large");
    const RecLayout R = rec_layout(c, nsteps, ckpt_every);
    sizes[0] = R.total;
    sizes[1] = R.total_seg;
    sizes[2] = R.total_all;
    return ABM_OK;
}

int abm_record_info(abm_ctx* c, int32_t* info) {
    if (int rc = check_ctx(c)) return rc;
    if (!info) return fail(ABM_E_INVAL, "null output");
    info[0] = c->recorded ? c->rec_tapes : -1;
    info[1] = c->taped_reverse;
    info[2] = int32_t(std::min<uint32_t>(c->rec_worst, 0x7FFFFFFFu));
    return ABM_OK;
}

int abm_forward_record(abm_ctx* c, int32_t nsteps, int32_t ckpt_every, void* rec, int64_t rec_bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps < 1 || ckpt_every < 1 || !rec) return fail(ABM_E_INVAL, "bad arguments");
    if (!record_fits(c, nsteps)) return fail(ABM_E_INVAL, "record too large");
    if (c->nsims != 1) return fail(ABM_E_UNSUPPORTED, "the adjoint covers a single simulation");
    if (c->params.detect_static) return fail(ABM_E_UNSUPPORTED, "the adjoint needs detect_static off");
    if (reinterpret_cast<uintptr_t>(rec) % kAlign) return fail(ABM_E_INVAL, "record buffer must be 256-byte aligned");
    return c->precision == ABM_F64 ? forward_record_impl<double>(c, nsteps, ckpt_every, rec, rec_bytes)
                                   : forward_record_impl<float>(c, nsteps, ckpt_every, rec, rec_bytes);
}

int abm_backward(abm_ctx* c, const void* dL_dxT, void* dL_dx0, void* dL_dparams) {
    if (int rc = check_ctx(c)) return rc;
    if (!dL_dxT || !dL_dx0 || !dL_dparams) return fail(ABM_E_INVAL, "null argument");
    const double* a = static_cast<const double*>(dL_dxT);
    double* b = static_cast<double*>(dL_dx0);
    double* p = static_cast<double*>(dL_dparams);
    return c->precision == ABM_F64 ? backward_impl<double>(c, a, b, p) : backward_impl<float>(c, a, b, p);
}

int abm_set_timing(abm_ctx* c, int32_t enable) {
    if (int rc = check_ctx(c)) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& e : c->ev_pending) c->ev_free.push_back(e);
    c->ev_pending.clear();
    for (double& m : c->ev_ms) m = 0.0;
    c->ev_steps = 0;
    c->timing = enable == 2 ? 2 : (enable != 0 ? 1 : 0);
    return ABM_OK;
}

int abm_get_timing(abm_ctx* c, abm_timing* out) {
    if (int rc = check_ctx(c)) return rc;
    if (!out) return fail(ABM_E_INVAL, "null output");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& e : c->ev_pending) {
        // the pending steps all have the mode they were timed in (setting it
        // drops them)
        for (int k = c->timing == 2 ? kTimedPhases - 1 : 0; k < kTimedPhases; ++k) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e[k], e[k + 1]));
            c->ev_ms[k] += ms;
        }
        c->ev_steps += 1;
        c->ev_free.push_back(e);
    }
    c->ev_pending.clear();
    out->steps = c->ev_steps;
    for (int k = 0; k < kTimedPhases; ++k) out->ms[k] = c->ev_ms[k];
    for (int k = kTimedPhases; k < 8; ++k) out->ms[k] = 0.0;
    return ABM_OK;
}

void abm_destroy(abm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto* v : {&c->ev_pending, &c->ev_free})
        for (auto& e : *v)
            for (auto& x : e) (void)hipEventDestroy(x);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->ws = nullptr;
    delete c;
}

}  // extern "C"
