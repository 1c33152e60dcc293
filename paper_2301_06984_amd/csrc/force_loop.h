// force_loop.h -- the neighbour walk and the pair force, shared by the step
// kernel and the reverse-mode kernels.
//
// The walk reads the agents of a super-box from the grid's loose position
// array ({x, y, z, d}, sign of d = moved in the last step) at the slot range
// its table entry gives.  The walk covers the 3x3x3 boxes of Section 3.1 through
// super-boxes, the aligned 2x2x2 blocks S = q >> 1 of boxes: a super-box is 8
// consecutive Morton codes, so its agents are one contiguous slot range,
// sorted by octant.  Along each axis the boxes q-1..q+1 lie in two
// super-boxes, so 8 super-boxes hold the 27 boxes.  Of one of the two along
// an axis only one half is needed; the super-box table keeps the agent
// counts at the octant boundaries 2, 4 and 6, so the y and z halves that are
// not needed are cut off where that leaves one slot range per super-box
// (z halves always, y halves when z is cut too), leaving at most 8 slot
// ranges ("pieces") over 4 x 3 x 3 boxes plus two 2 x 1 x 2 blocks.  Agents
// of the boxes outside the 27 are rejected by the distance test like any
// other non-neighbour.
//
// The 8 super-boxes are visited in Morton order, which is slot order, without
// sorting: two super-boxes of the 2x2x2 block that differ along a set of axes
// compare by the highest interleaved bit in which their codes differ, and for
// axis a that is bit 3 t_a + a, t_a the number of trailing one bits of the
// block's lower coordinate on that axis.  So the block's Morton order is a
// 3-bit count whose digits are the axes ranked by 3 t_a + a.  Pieces within a
// super-box are in octant order, hence the walk yields every neighbour in
// canonical (box rank, id) order, the order of the sums, wherever the grid
// put each super-box's slot range.
#pragma once

#include "abm_device.h"

namespace abm {

template <class T>
__device__ __forceinline__ const V4<T>* gpos_ptr(const Buffers<T>& b) {
    return reinterpret_cast<const V4<T>*>(b.gpos);
}

// Super-box table entry (16 B):
//   x  first loose slot of the super-box
//   y  number of its agents (bits 0..23); bit 24 + o: an agent of octant o
//      moved in the last step
//   z  agents in octants < 2 (bits 0..15) and in octants < 4 (bits 16..31)
//   w  agents in octants < 6 (bits 0..15), 15-bit stamp of the step that
//      wrote the entry (bits 17..31)
// With more than kMaxSplitCount agents the octant counts are not kept and
// the whole range is walked; kMaxSuperCount agents is the limit (grid error
// beyond).
constexpr uint32_t kMaxSplitCount = 0xFFFFu;
constexpr uint32_t kMaxSuperCount = 0xFFFFFFu;

__device__ __forceinline__ uint4 pack_super(uint32_t start, uint32_t total, uint32_t c2, uint32_t c4, uint32_t c6,
                                            uint32_t moved_octants, uint32_t stamp) {
    if (total > kMaxSplitCount) c2 = c4 = c6 = 0u;
    return make_uint4(start, (total & kMaxSuperCount) | (moved_octants << 24), (c2 & 0xFFFFu) | (c4 << 16),
                      (c6 & 0xFFFFu) | ((stamp & 0x7FFFu) << 17));
}
__device__ __forceinline__ uint32_t super_stamp(const uint4& e) { return e.w >> 17; }

__device__ __forceinline__ uint32_t super_dim(uint32_t d) { return (d + 1u) >> 1; }

// Global index of super-box (sx, sy, sz) in the row-major table.
__device__ __forceinline__ uint32_t super_index(const SimGrid& G, uint32_t sx, uint32_t sy, uint32_t sz) {
    return G.sbase + (sz * G.sdims[1] + sy) * G.sdims[0] + sx;
}

// Box coordinates of a position relative to the simulation's grid.
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

// Per-thread scratch in LDS for the neighbour walk: the pieces (start slot in
// the low, end slot in the high 32 bits) and a queue of candidate slots.  Laid
// out [entry][thread] so that the threads of a wave hit distinct banks.
// LDS per thread of the walk: kPieces * 8 + queue_cap<CH>() * 4 bytes,
// which bounds the waves per CU.  The walk tests CH = 2 or 4 candidate slots
// of a piece together (4 pays off where boxes hold many agents).
constexpr int kPieces = 8;   // one per super-box of the 2x2x2 block, in Morton order
// Queue rows of a lane.  A lane whose queue fills mid-walk runs the exact test
// (and its own pair terms) alone while the rest of its wave waits.  The 2-wide
// walk takes 14 rows: an agent with a few dozen candidates (uniform packing)
// then finishes its walk first, so that one exact test serves the whole wave,
// and five blocks of 256 threads still fit a CU.  The 4-wide walk (clustered
// agents, thousands of candidates, whose queues fill whatever their depth)
// takes 5, the least a chunk of 4 needs: every lane then flushes after nearly
// every chunk, so the lanes of a wave flush together.
template <int CH>
constexpr int queue_cap() { return CH == 2 ? 14 : 5; }
static_assert(4 <= kSposPad, "the walk reads up to 3 slots past a piece");
struct WalkLds {
    unsigned long long* rng;   // [kPieces][blockDim]
    uint32_t* queue;           // [queue_cap<CH>()][blockDim]
};
template <int CH>
inline size_t walk_lds_bytes(int block) { return size_t(block) * (kPieces * 8 + queue_cap<CH>() * 4); }

__device__ __forceinline__ WalkLds walk_lds(void* base) {
    WalkLds w;
    w.rng = static_cast<unsigned long long*>(base);
    w.queue = reinterpret_cast<uint32_t*>(w.rng + kPieces * blockDim.x);
    return w;
}

struct Pieces {
    uint32_t mask = 0;    // bit j: piece j (Morton position j of its super-box) is not empty
    uint32_t total = 0;   // slots in all pieces
    uint32_t xown = 0;    // first loose slot of the super-box of box q
    bool moved = false;   // an agent of one of the 27 boxes moved in the last step
};

// The slot range [a0, a1) (offsets from the first slot) of the part of a
// super-box with table entry e that a piece takes: all of it, or with
// ty (tz) only its y (z) half hy (hz), where the octant counts allow one
// contiguous range: z halves always, a y half inside a z half, and with y
// cut but z not, octants 2 hy .. 2 hy + 5.  Super-boxes of more than
// kMaxSplitCount agents are taken whole.
__device__ __forceinline__ void trim_range(const uint4& e, bool ty, bool tz, uint32_t hy, uint32_t hz, uint32_t* a0,
                                           uint32_t* a1) {
    const uint32_t c8 = e.y & kMaxSuperCount, c2 = e.z & 0xFFFFu, c4 = e.z >> 16, c6 = e.w & 0xFFFFu;
    const bool split = c8 <= kMaxSplitCount;
    ty = ty && split;
    tz = tz && split;
    // octant count bounds of the needed y half in the lower (z bit 0) and
    // the upper (z bit 1) layer of the super-box
    const uint32_t ylo0 = hy ? c2 : 0u, yhi0 = hy ? c4 : c2;
    const uint32_t ylo1 = hy ? c6 : c4, yhi1 = hy ? c8 : c6;
    uint32_t b0 = 0u, b1 = c8;
    if (tz) {
        b0 = ty ? (hz ? ylo1 : ylo0) : (hz ? c4 : 0u);
        b1 = ty ? (hz ? yhi1 : yhi0) : (hz ? c8 : c4);
    } else if (ty) {   // y cut, z not: one piece over octants 2h..2h+5
        b0 = ylo0;
        b1 = yhi1;
    }
    *a0 = b0;
    *a1 = b1;
}

// Load the pieces around box q (entries of the current stamp only) into this
// thread's LDS rows, piece j at row j.  The super-boxes are visited in
// row-major order, so that their table offsets and range tests are fixed
// per visit; each writes its piece at its Morton position.
template <class T>
__device__ __forceinline__ Pieces load_pieces(const Buffers<T>& b, const SimGrid& G, const uint32_t q[3],
                                              uint32_t stamp, const WalkLds& L) {
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    const uint32_t sd0 = G.sdims[0], sd1 = G.sdims[1], sd2 = G.sdims[2];
    uint32_t lo[3], bq[3], rank_key[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bq[a] = q[a] & 1u;
        lo[a] = (q[a] >> 1) - 1u + bq[a];   // wraps below 0: then out of range
        rank_key[a] = 3u * uint32_t(__builtin_ctz(~lo[a] | 0x80000000u)) + uint32_t(a);
    }
    // weight of each axis in the Morton position of a super-box of the block
    const uint32_t wx = 1u << ((rank_key[0] > rank_key[1] ? 1u : 0u) + (rank_key[0] > rank_key[2] ? 1u : 0u));
    const uint32_t wy = 1u << ((rank_key[1] > rank_key[0] ? 1u : 0u) + (rank_key[1] > rank_key[2] ? 1u : 0u));
    const uint32_t wz = 1u << ((rank_key[2] > rank_key[0] ? 1u : 0u) + (rank_key[2] > rank_key[1] ? 1u : 0u));
    const bool inx[2] = {lo[0] < sd0, lo[0] + 1u < sd0};
    const bool iny[2] = {lo[1] < sd1, lo[1] + 1u < sd1};
    const bool inz[2] = {lo[2] < sd2, lo[2] + 1u < sd2};
    const uint32_t plane = sd0 * sd1;
    const uint32_t base = G.sbase + (lo[2] * sd1 + lo[1]) * sd0 + lo[0];   // modulo 2^32; exact when in range
    const uint32_t st15 = stamp & 0x7FFFu;
    const uint32_t hy = bq[1] ^ 1u, hz = bq[2] ^ 1u;   // the half needed of a trimmed super-box
    // octants of the super-box at offset d (per axis) that hold boxes of the
    // 3x3x3 block: all, or only the half on the near side
    const uint32_t xm[2] = {bq[0] ? 0xFFu : 0xAAu, bq[0] ? 0x55u : 0xFFu};
    const uint32_t ym[2] = {bq[1] ? 0xFFu : 0xCCu, bq[1] ? 0x33u : 0xFFu};
    const uint32_t zm[2] = {bq[2] ? 0xFFu : 0xF0u, bq[2] ? 0x0Fu : 0xFFu};
    uint32_t moved = 0;
    Pieces P;
    const int own = int(bq[0] ^ 1u) | int((bq[1] ^ 1u) << 1) | int((bq[2] ^ 1u) << 2);   // S = q >> 1
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t dx = uint32_t(c) & 1u, dy = (uint32_t(c) >> 1) & 1u, dz = uint32_t(c) >> 2;
        uint4 e = make_uint4(0u, 0u, 0u, 0u);
        if (inx[dx] && iny[dy] && inz[dz]) e = b.cellinfo[base + dz * plane + dy * sd0 + dx];
        if (super_stamp(e) != st15) e = make_uint4(0u, 0u, 0u, 0u);
        P.xown = c == own ? e.x : P.xown;
        moved |= (e.y >> 24) & xm[dx] & ym[dy] & zm[dz];
        // the y (z) half of this super-box is cut when it lies on the far side
        uint32_t a0, a1;
        trim_range(e, dy == bq[1], dz == bq[2], hy, hz, &a0, &a1);
        const uint32_t j = dx * wx + dy * wy + dz * wz;
        L.rng[j * bs + tid] = (unsigned long long)(e.x + a0) | ((unsigned long long)(e.x + a1) << 32);
        P.mask |= (a1 > a0 ? 1u : 0u) << j;
        P.total += a1 - a0;
    }
    P.moved = moved != 0u;
    return P;
}

// The slots of the pieces as one stream in ascending order; a wave iterates
// max(total) times rather than the sum of per-piece maxima.  fn(slot)
// returns false to stop; stream_pieces then returns false.
template <class Fn>
__device__ __forceinline__ bool stream_pieces(const WalkLds& L, const Pieces& P, Fn&& fn) {
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    uint32_t M = P.mask;
    if (!M) return true;
    uint32_t k = uint32_t(__ffs(M)) - 1u;
    M &= M - 1u;
    unsigned long long v = L.rng[k * bs + tid];
    uint32_t u = uint32_t(v), e = uint32_t(v >> 32);
    for (;;) {
        if (!fn(u)) return false;
        if (++u == e) {
            if (!M) break;
            k = uint32_t(__ffs(M)) - 1u;
            M &= M - 1u;
            v = L.rng[k * bs + tid];
            u = uint32_t(v);
            e = uint32_t(v >> 32);
        }
    }
    return true;
}

// The pieces CH slots at a time, with the positions of the next chunk
// requested before the current one is tested (two register buffers, A and B,
// take turns).  A chunk is [u, u + CH) of a piece [.., e); the next
// non-empty piece is already read from LDS.  Slots past the piece end are
// read (the loose position array is padded) but must not be used:
// test(pc, u, left) sees the chunk's positions, its first slot and the
// number of its slots inside the piece, and returns false to stop the walk.
//
// sp is the position source the pieces index: the grid's loose position
// array, or a block's copy of its neighbourhood in LDS.
template <int CH, class T, class Test>
__device__ __forceinline__ void walk_chunks(const V4<T>* __restrict__ sp, const Pieces& P, const WalkLds& L,
                                            Test&& test) {
    static_assert(CH >= 1 && CH <= kSposPad && queue_cap<CH>() > CH, "walk chunk");
    if (!P.mask) return;
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    uint32_t M = P.mask;
    const uint32_t k0 = uint32_t(__ffs(M)) - 1u;
    M &= M - 1u;
    const unsigned long long v0 = L.rng[k0 * bs + tid];
    unsigned long long nxt = L.rng[(M ? uint32_t(__ffs(M)) - 1u : k0) * bs + tid];
    const uint32_t safe = uint32_t(v0);   // a slot whose chunk lies in the array
    // move (uu, ee) to the chunk after it; false at the end of the stream
    auto advance = [&](uint32_t& uu, uint32_t& ee) -> bool {
        uu += CH;
        if (uu < ee) return true;
        if (!M) return false;
        uu = uint32_t(nxt);
        ee = uint32_t(nxt >> 32);
        M &= M - 1u;
        if (M) nxt = L.rng[(uint32_t(__ffs(M)) - 1u) * bs + tid];
        return true;
    };
    auto fetch = [&](V4<T>* pc, uint32_t uu, bool has) {
        const V4<T>* __restrict__ pu = sp + (has ? uu : safe);
#pragma unroll
        for (int c = 0; c < CH; ++c) pc[c] = pu[c];
    };
    V4<T> pa[CH], pb[CH];
    uint32_t ua = uint32_t(v0), ea = uint32_t(v0 >> 32);
    fetch(pa, ua, true);
    uint32_t ub = ua, eb = ea;
    bool hb = advance(ub, eb);
    fetch(pb, ub, hb);
    for (;;) {
        if (!test(pa, ua, ea - ua) || !hb) break;
        ua = ub;
        ea = eb;
        const bool ha = advance(ua, ea);
        fetch(pa, ua, ha);
        if (!test(pb, ub, eb - ub) || !ha) break;
        ub = ua;
        eb = ea;
        hb = advance(ub, eb);
        fetch(pb, ub, hb);
    }
}

// Conservative single-precision pre-test of |x_i - x_j|^2 < R^2: false only
// if the exact double test must fail.  The float sum of squares is within a
// few ulp (relative) of the exact value: for float state the differences are
// float roundings of the exact ones, for double state float roundings of the
// double differences (about 5 * 2^-24 relative in all, far inside the 2^-16
// relative padding of the bound; a difference too large for float becomes
// infinite and fails, as the exact test does).
template <class T>
__device__ __forceinline__ bool maybe_within(const V4<T>& pi, const V4<T>& pj, float r2pad) {
    if constexpr (sizeof(T) == 4) {
        const float ex = pi.x - pj.x, ey = pi.y - pj.y, ez = pi.z - pj.z;
        return __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)) < r2pad;
    } else {
        const float ex = float(pi.x - pj.x), ey = float(pi.y - pj.y), ez = float(pi.z - pj.z);
        return __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)) < r2pad;
    }
}

__device__ __forceinline__ float padded_r2(double r2) { return float(r2 * (1.0 + 1.0 / 65536.0)) * 1.0001f; }

struct ForceSum {
    double fx = 0.0, fy = 0.0, fz = 0.0;   // F_i
    double kx = 0.0, ky = 0.0, kz = 0.0;   // dF_i/dk    = sum_j delta_ij u_ij
    double gx = 0.0, gy = 0.0, gz = 0.0;   // dF_i/dgamma = -sum_j sqrt(rho_ij delta_ij) u_ij
    uint32_t nnz = 0;
    bool moved_near = false;               // an agent within R (not i) moved in the last step
};

// One pair term: f = k delta - gamma sqrt(rho delta) along e / |e| (the
// force-law reading of Section 5), for agent i at (xi, yi, zi) with radius ri
// and a neighbour pj in contact.  Evaluated in double, without fused
// multiply-adds (the library is built with contraction off).
struct PairTerm {
    double fx, fy, fz;      // the term's force on i
    double delta, sr, dist; // overlap, sqrt(rho delta), |e|
    double ex, ey, ez;
    bool nonzero;
};
template <class T>
__device__ __forceinline__ PairTerm pair_term(double xi, double yi, double zi, double ri, const V4<T>& pj, double k,
                                              double gamma) {
    PairTerm t;
    t.ex = xi - double(pj.x);
    t.ey = yi - double(pj.y);
    t.ez = zi - double(pj.z);
    const double s2 = (t.ex * t.ex + t.ey * t.ey) + t.ez * t.ez;
    const double rj = 0.5 * fabs(double(pj.w));
    const double S = ri + rj;
    t.dist = sqrt(s2);
    t.delta = S - t.dist;
    const double rho = (ri * rj) / S;
    t.sr = sqrt(rho * t.delta);
    const double f = k * t.delta - gamma * t.sr;
    const double sc = f / t.dist;
    t.fx = sc * t.ex;
    t.fy = sc * t.ey;
    t.fz = sc * t.ez;
    t.nonzero = f != 0.0;
    return t;
}

// Adds one pair term to F_i (and, with PARAM_GRADS, to dF_i/dk and
// dF_i/dgamma); every walk that sums pair terms adds them through this.
template <bool PARAM_GRADS>
__device__ __forceinline__ void add_term(ForceSum& acc, const PairTerm& t) {
    acc.fx += t.fx;
    acc.fy += t.fy;
    acc.fz += t.fz;
    acc.nnz += t.nonzero ? 1u : 0u;
    if (PARAM_GRADS) {
        const double ux = t.ex / t.dist, uy = t.ey / t.dist, uz = t.ez / t.dist;
        acc.kx += t.delta * ux;
        acc.ky += t.delta * uy;
        acc.kz += t.delta * uz;
        acc.gx -= t.sr * ux;
        acc.gy -= t.sr * uy;
        acc.gz -= t.sr * uz;
    }
}

// F_i over the neighbours j (|e|^2 < R^2) in contact (0 < |e| < r_i + r_j),
// summed in ascending slot order.
//
// Pass 1 takes the candidates CH slots of one piece at a time (their
// positions requested together) through the cheap pre-test and queues the
// survivors (the agent itself among them: the exact test drops d = 0).  A
// nearly full queue is compacted by the exact test (neighbour and contact,
// in place), which keeps the contacts in slot order at its head.
//
// The pair terms: without SHARE, each lane adds its own contacts' terms when
// its queue fills and at the end.  With SHARE, force_of is entered by every
// lane of the wave; a lane adds its contacts itself only if they fill its
// queue, and at the end the wave shares out all its lanes' remaining
// contacts, one per lane, and each term goes back to its agent's lane by
// register shuffles (the j-th term of every lane at once), which adds them in
// slot order: the same sums, bit for bit, with the lanes of a wave busy
// however unevenly the contacts fall.
//
// sp is the position source the pieces and queue rows index, last its last
// readable index.  emit(k) sees each batch of contacts, queue rows [0, k),
// before their terms are added: all of them, in the order they are summed.
struct NoEmit {
    __device__ __forceinline__ void operator()(uint32_t) const {}
};
template <int CH, class T, bool PARAM_GRADS, bool SHARE = false, class Emit = NoEmit>
__device__ __forceinline__ void force_of(const V4<T>* __restrict__ sp, const uint32_t last, const SimGrid& G,
                                         const V4<T>& p, const Pieces& P, const WalkLds& L, ForceSum& acc,
                                         Emit emit = Emit{}) {
    static_assert(!(SHARE && PARAM_GRADS), "shared pair terms carry the force only");
    constexpr int QC = queue_cap<CH>();
    const uint32_t tid = threadIdx.x, bs = blockDim.x;
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double ri = 0.5 * fabs(double(p.w));
    const double r2 = G.r2, k = G.k, gamma = G.gamma;
    const float r2pad = padded_r2(r2);
    uint32_t n = 0;      // queue rows in use
    uint32_t kept = 0;   // rows [0, kept): contacts whose terms are not added yet
    // exact neighbour + contact test of rows [kept, n), keeping the contacts
    // in place after row kept; the positions of a group of four are
    // requested before any is tested
    auto exact = [&]() {
        uint32_t m = kept;
        for (uint32_t x0 = kept; x0 < n; x0 += 4) {
            V4<T> pj[4];
            uint32_t uq[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uq[c] = L.queue[min(x0 + c, n - 1) * bs + tid];
                pj[c] = sp[min(uq[c], last)];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double ex = xi - double(pj[c].x), ey = yi - double(pj[c].y), ez = zi - double(pj[c].z);
                const double s2 = (ex * ex + ey * ey) + ez * ez;
                const double S = ri + 0.5 * fabs(double(pj[c].w));
                const bool within = x0 + c < n && s2 < r2;
                // the sign of d carries the moved flag (the agent itself counts
                // only where this feeds a static test, and then it did not move)
                acc.moved_near = acc.moved_near || (within && pj[c].w < T(0));
                const bool keep = within && s2 > 0.0 && s2 < S * S;
                // only rows in use are rewritten: with every tested row kept,
                // m reaches n, and n can be QC, one row past the queue
                if (x0 + c < n) L.queue[m * bs + tid] = uq[c];
                m += keep ? 1u : 0u;
            }
        }
        kept = m;
        n = m;
    };
    // this lane's contacts, rows [0, kept), in order; four positions requested together
    auto own_terms = [&]() {
        emit(kept);
        for (uint32_t x0 = 0; x0 < kept; x0 += 4) {
            V4<T> pj4[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) pj4[c] = sp[min(L.queue[min(x0 + c, kept - 1) * bs + tid], last)];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (x0 + c >= kept) break;
                add_term<PARAM_GRADS>(acc, pair_term<T>(xi, yi, zi, ri, pj4[c], k, gamma));
            }
        }
        kept = 0;
        n = 0;
    };
    // pass 1: the pre-test over the walk, survivors queued in slot order
    uint32_t qo = tid;   // this thread's next queue entry
    walk_chunks<CH, T>(sp, P, L, [&](const V4<T>* pc, uint32_t u, uint32_t left) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            // no short-circuit: every lane does the same arithmetic
            const uint32_t pass = uint32_t(uint32_t(c) < left) & uint32_t(maybe_within<T>(p, pc[c], r2pad));
            L.queue[qo] = u + c;   // n < QC here
            n += pass;
            qo += pass ? bs : 0u;
        }
        if (n > uint32_t(QC - CH)) {
            exact();
            if (!SHARE || n > uint32_t(QC - CH)) own_terms();
            qo = n * bs + tid;
        }
        return true;
    });
    exact();
    if constexpr (!SHARE) {
        own_terms();
    } else {
        emit(kept);
        // the wave's contacts: lane l's rows [0, kept) are pairs [off, off +
        // kept) of the wave, pair x evaluated by lane x mod 64 in round x / 64
        const uint32_t lane = uint32_t(lane_id()), wbase = tid - lane;
        uint32_t incl = kept;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, 64);
            if (lane >= uint32_t(d)) incl += y;
        }
        const uint32_t off = incl - kept, total = __shfl(incl, 63, 64);
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t x = base + lane;
            // the pair's agent: the last lane whose pairs start at or before x
            uint32_t o = 0;
            for (uint32_t step = 32; step >= 1; step >>= 1) {
                const uint32_t v = __shfl(off, int(o + step), 64);
                o = v <= x ? o + step : o;
            }
            const uint32_t row = x - __shfl(off, int(o), 64);
            const double oxi = __shfl(xi, int(o), 64), oyi = __shfl(yi, int(o), 64), ozi = __shfl(zi, int(o), 64);
            const double ori = __shfl(ri, int(o), 64), ok_ = __shfl(k, int(o), 64), og = __shfl(gamma, int(o), 64);
            PairTerm t{};
            t.fx = t.fy = t.fz = 0.0;
            t.nonzero = false;
            if (x < total) {
                const uint32_t uj = L.queue[min(row, uint32_t(QC - 1)) * bs + wbase + o];
                t = pair_term<T>(oxi, oyi, ozi, ori, sp[min(uj, last)], ok_, og);
            }
            const unsigned long long nzm = __ballot(x < total && t.nonzero);
            // this lane's pairs in the round: [lo, hi) of the wave's numbering
            const uint32_t lo = max(off, base), hi = min(off + kept, base + 64u);
            if (hi > lo) {
                const uint32_t a0 = lo - base, a1 = hi - base;
                const unsigned long long bits = (a1 >= 64u ? ~0ull : ((1ull << a1) - 1ull)) & ~((1ull << a0) - 1ull);
                acc.nnz += uint32_t(__popcll(nzm & bits));
            }
            // the terms go back to their agent's lane: the j-th of every lane at once
            const uint32_t j0 = max(off, base), j1 = min(off + kept, base + 64u);
            const uint32_t cnt = j1 > j0 ? j1 - j0 : 0u;
            uint32_t most = cnt;
            for (int d = 32; d >= 1; d >>= 1) most = max(most, uint32_t(__shfl_xor(int(most), d, 64)));
            for (uint32_t j = 0; j < most; ++j) {
                const int src = int(min(j0 + j - base, 63u));
                const double vx = __shfl(t.fx, src, 64), vy = __shfl(t.fy, src, 64), vz = __shfl(t.fz, src, 64);
                if (j < cnt) {
                    acc.fx += vx;
                    acc.fy += vy;
                    acc.fz += vz;
                }
            }
        }
    }
}

// force_of over the grid's loose position array.
template <int CH, class T, bool PARAM_GRADS, bool SHARE = false, class Emit = NoEmit>
__device__ __forceinline__ void force_of(const Buffers<T>& b, const SimGrid& G, const V4<T>& p, const Pieces& P,
                                         const WalkLds& L, ForceSum& acc, Emit emit = Emit{}) {
    force_of<CH, T, PARAM_GRADS, SHARE, Emit>(gpos_ptr(b), 2u * b.n - 1u, G, p, P, L, acc, emit);
}

// The walk's pre-test and exact test for agent p, keeping its contacts
// (neighbours within R, 0 < |e| < r_i + r_j) at the head of its LDS queue in
// slot order; returns their number, rows [0, kept).  When contacts fill the
// queue mid-walk, own(kept) consumes rows [0, kept) first.
template <int CH, class T, class Own>
__device__ __forceinline__ uint32_t queue_contacts(const Buffers<T>& b, const SimGrid& G, const V4<T>& p,
                                                   const Pieces& P, const WalkLds& L, Own&& own) {
    const V4<T>* __restrict__ sp = gpos_ptr(b);
    constexpr int QC = queue_cap<CH>();
    const uint32_t tid = threadIdx.x, bs = blockDim.x, last = 2u * b.n - 1u;
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    const double ri = 0.5 * fabs(double(p.w));
    const double r2 = G.r2;
    const float r2pad = padded_r2(r2);
    uint32_t n = 0, kept = 0;
    // exact test of rows [kept, n), the contacts kept in place after row kept
    auto exact = [&]() {
        uint32_t m = kept;
        for (uint32_t x0 = kept; x0 < n; x0 += 4) {
            V4<T> pj[4];
            uint32_t uq[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uq[c] = L.queue[min(x0 + c, n - 1) * bs + tid];
                pj[c] = sp[min(uq[c], last)];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double ex = xi - double(pj[c].x), ey = yi - double(pj[c].y), ez = zi - double(pj[c].z);
                const double s2 = (ex * ex + ey * ey) + ez * ez;
                const double S = ri + 0.5 * fabs(double(pj[c].w));
                const bool keep = x0 + c < n && s2 < r2 && s2 > 0.0 && s2 < S * S;
                if (x0 + c < n) L.queue[m * bs + tid] = uq[c];   // rows in use only (see force_of)
                m += keep ? 1u : 0u;
            }
        }
        kept = m;
        n = m;
    };
    uint32_t qo = tid;
    walk_chunks<CH, T>(sp, P, L, [&](const V4<T>* pc, uint32_t u, uint32_t left) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const uint32_t pass = uint32_t(uint32_t(c) < left) & uint32_t(maybe_within<T>(p, pc[c], r2pad));
            L.queue[qo] = u + c;   // n < QC here
            n += pass;
            qo += pass ? bs : 0u;
        }
        if (n > uint32_t(QC - CH)) {
            exact();
            if (kept > uint32_t(QC - CH)) {
                own(kept);
                kept = n = 0;
            }
            qo = n * bs + tid;
        }
        return true;
    });
    exact();
    return kept;
}

// Displacement rule: Delta = mu F if |F| > f_adh, clamped to delta_max.
struct Move {
    double ux = 0.0, uy = 0.0, uz = 0.0;
    bool moves = false;
    bool clamped = false;
    double fnorm = 0.0;
    double size = 0.0;   // |Delta|: |mu F|, or delta_max where clamped
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
        m.size = un;
        if (un > G.delta_max) {
            m.size = G.delta_max;
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
