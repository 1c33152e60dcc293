// force_kernels.hip -- static flags, pair forces, displacement and the
// Jacobi commit of one step (Section 5, Algorithm 1), plus the copies that
// move per-agent fields in and out of the internal layout.
#include "force_loop.h"

namespace abm {

// Simulations whose box extents one block of the step kernel folds in LDS
// (further ones, in blocks spanning many small simulations, go straight to
// the global accumulators).
constexpr int kMaxBlockSims = 4;

// One thread per loose slot of the grid (Section 4.2, step G): the agents of
// a super-box sit in consecutive slots in canonical order, so a wave works on
// agents that are close in space and shares their neighbour boxes in cache.
// Chunks of blockDim slots: nb = ceil(n / blockDim) chunks cover the
// storage slots [0, n) (agents there only in an update build, and not in
// slots marked dead), nb more the append region [n, n + napp).  With the
// 2-wide walk, block k takes append chunk k and storage chunk k, those that
// hold agents (nb blocks, two copies of the agent code); with the 4-wide walk
// (more registers), each block takes one chunk, append chunks after storage
// chunks, and a launch for a full build starts at the append chunks; a block
// whose chunks hold no agent returns at once.  The agent's storage index is i = u below n,
// else perm[u - n].  The new state goes to storage index i, or, when this
// step re-lays agents out in Morton order, to the agent's canonical slot: its
// super-box's start plus its offset in the super-box's loose range; the step
// then also writes the ids and grid keys in that order, which lets the next
// grid be built as an update.  The static test (Section 5) runs first: an
// agent that did not move, had at most one non-zero pair term, and has no
// moved neighbour within R keeps its force and does not move.  The new
// positions' box extent is reduced here for the next step's grid: each wave
// folds into the block's LDS copy, and the block's last wave to finish adds
// it to the global accumulators, so no wave waits for the others.
// With TAPE (one simulation, static test off, a full build), the step also
// writes its contact tape: each agent's contacts, in the order their terms
// are summed, with its position and id, by canonical slot (the adjoint's
// reverse step reads it instead of walking a grid).
// At 96 VGPRs or fewer a SIMD holds 5 waves of this kernel (4 above); the
// hint asks the compiler for 5 in FP32 state.  In FP64 state the positions
// take twice the registers: held to 5 waves the kernel spills 20-140 bytes
// per lane, at 4 it spills less and runs 5-10% faster.
template <class T>
constexpr int force_waves_per_eu() { return sizeof(T) == 8 ? 4 : 5; }
template <int CH>
constexpr bool two_chunks() { return CH == 2; }

template <class T, bool BATCHED, bool STATIC_ON, bool RELAYOUT, int CH, bool TAPE = false, bool SHARE = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(force_waves_per_eu<T>()))) void k_force(
    Buffers<T> b, StepArgs a, uint32_t run, uint32_t first_chunk) {
    static_assert(!TAPE || (!BATCHED && !STATIC_ON), "tapes cover the adjoint's steps only");
    extern __shared__ __align__(16) unsigned char s_walk[];
    __shared__ int32_t s_box[kMaxBlockSims][6];
    __shared__ int s_sims[kMaxBlockSims];
    __shared__ uint32_t s_cnt[3];   // static, moved, waves done
    __shared__ double s_fsum[16][3];            // per wave: sum of the forces it evaluated
    __shared__ unsigned long long s_dmax[16];   // per wave: largest displacement (ordered bits)
    const uint32_t n = b.n, bs = blockDim.x, nb = (n + bs - 1) / bs;
    const uint32_t napp = min(b.g->napp, n);
    const bool inc = b.g->inc != 0u;
    // the block's chunks: append chunk ka and storage chunk ks, where they hold agents
    uint32_t ka = 0, ks = 0;
    bool has_a = false, has_s = false;
    if constexpr (two_chunks<CH>()) {
        ka = ks = xcd_block(run);
        has_a = ka * bs < napp;
        has_s = inc && ks < nb;
    } else {
        const uint32_t chunk = first_chunk + xcd_block(run);
        ka = chunk - nb;
        ks = chunk;
        has_a = chunk >= nb && ka * bs < napp;
        has_s = chunk < nb && inc;
    }
    if (!has_a && !has_s) {   // no agent in the block's chunks
        if (!BATCHED && threadIdx.x == 0)
            b.bpart[blockIdx.x] =
                BlockPart{{INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN}, 0u, 0u, {0.0, 0.0, 0.0}, 0ull};
        return;
    }
    const WalkLds L = walk_lds(s_walk);
    // the block's agents mostly belong to at most kMaxBlockSims simulations
    // from that of its chunk's first slot on (others fold straight into the
    // global accumulators); their LDS accumulators start empty
    const int sim0 = BATCHED ? sim_index(b, min((has_a ? ka : ks) * bs, n - 1u)) : 0;
    if (threadIdx.x < kMaxBlockSims * 6) {
        const int k = int(threadIdx.x) % 6;
        s_box[threadIdx.x / 6][k] = k < 3 ? INT32_MAX : INT32_MIN;
    }
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0u;
    if (threadIdx.x < kMaxBlockSims) s_sims[threadIdx.x] = -1;
    if (threadIdx.x < 16) {
        for (int c = 0; c < 3; ++c) s_fsum[threadIdx.x][c] = 0.0;
        s_dmax[threadIdx.x] = 0ull;
    }
    __syncthreads();
    const int cur = a.pos_cur, nxt = cur ^ 1;
    const bool KEEP_F = a.keep_forces;
    // the agents of one chunk (c0 its first slot)
    auto chunk_agents = [&](const uint32_t c0, const bool append) {
        const uint32_t u = c0 + threadIdx.x;
        // key: for the canonical slot of an agent of an update build; i: the
        // storage index (a full build's append slot n + t is canonical slot t,
        // in the same simulation's range as its storage index)
        uint32_t key = kDeadKey, i = u;
        bool active = false;
        // the slot's key, position and flags (and an appended agent's storage
        // index) are requested together, from the slot's range alone, and the
        // gathers that need only the key (its super-box's new start, a kept
        // agent's id) right after, so that the chain of dependent loads ahead
        // of the walk stays short
        const V4<T>* __restrict__ pin = pos4_ptr(b, cur);
        const bool inb = !append ? u < n : u - n < napp;
        V4<T> p0{};
        uint32_t f0 = 0;
        if (inb) {
            if (!append || inc) key = b.skey[cur][u];
            p0 = pin[u];
            f0 = b.flags[cur][u];
            if (!append) {
                active = key != kDeadKey;
            } else {
                i = u - n;
                active = true;
                if (inc || !RELAYOUT || KEEP_F) {
                    i = b.perm[u - n];
                    active = i < n;
                    if (!active) raise_error(b.g, kErrInternal);
                }
            }
        }
        uint32_t cs_key = 0, id_kept = 0;
        if (RELAYOUT && inc && active) {
            const uint32_t sk = key >> 3;
            if (sk < b.g->total_super) cs_key = a.cs[sk];
            if (!append) id_kept = b.ids[a.ids_cur][i];
        }
        bool ok = false, is_static = false, moved = false;
        double st_f[3] = {0.0, 0.0, 0.0};   // this agent's force, if evaluated, for the step's statistics
        unsigned long long st_d = 0ull;       // |Delta| as ordered bits
        int sim = 0;
        int32_t cnew[3] = {0, 0, 0};
        // ---- before the walk, per agent
        const SimGrid* Gp = b.sims;
        V4<T> p{};
        Pieces P;
        uint32_t f = 0, out = i;
        bool cand = false, walks = false;
        V4<T>* __restrict__ pout = pos4_ptr(b, nxt);
        if (active) {
            // one simulation: its parameters are the same for every lane
            sim = BATCHED ? sim_index(b, i) : 0;
            Gp = b.sims + sim;
            const SimGrid& G = *Gp;
            if (!G.valid) {
                // grid overflow (reported at sync): the agent keeps its state (a
                // full build copied it to loose slot n + i, and its id and key
                // to the next state)
                pout[i] = p0;
                b.flags[nxt][i] = f0 | kBoxChangedBit;
                if (KEEP_F)
                    for (int c = 0; c < 3; ++c) b.force[nxt][3 * size_t(i) + c] = b.force[cur][3 * size_t(i) + c];
                ok = box_coord(double(p0.x), G.inv_h, &cnew[0]) && box_coord(double(p0.y), G.inv_h, &cnew[1]) &&
                     box_coord(double(p0.z), G.inv_h, &cnew[2]);
            } else {
                p = p0;   // own state, sign of d = moved
                f = f0;
                uint32_t q[3];
                if (!box_of<T>(G, p, q)) raise_error(b.g, kErrInternal);
                P = load_pieces(b, G, q, G.stamp, L);
                if (RELAYOUT && !inc) {
                    out = u - n;
                } else if (RELAYOUT) {
                    const uint32_t sk = key >> 3;
                    out = sk < b.g->total_super ? cs_key + (u - P.xown) : n;
                    if (u < P.xown || out >= n) {
                        raise_error(b.g, kErrInternal);
                        out = i;
                    }
                    // an agent kept in place carries its id and key to the next
                    // state (the grid build wrote those of the append region);
                    // written before the walk, so that they need not live
                    // through it
                    if (!append) {
                        b.ids[a.ids_cur ^ 1][out] = id_kept;
                        b.skey[nxt][out] = key;
                    }
                }
                // Static test (Section 5): the agent did not move, had at most one
                // non-zero pair term, and no agent within R moved.  At step 0
                // every agent carries the moved bit, so none is static.  With no
                // moved agent in the 27 boxes it holds at once; otherwise the
                // force walk itself reports a moved agent within R.
                cand = STATIC_ON && !(f & kMovedBit) && (f >> kNnzShift) <= 1u;
                if (KEEP_F && cand)   // a static agent keeps its force (replaced below if it is not static)
                    for (int c = 0; c < 3; ++c) b.force[nxt][3 * size_t(out) + c] = b.force[cur][3 * size_t(i) + c];
                is_static = cand && !P.moved;
                p.w = T(fabs(double(p.w)));
                walks = !is_static;
            }
        }
        // ---- the walk and the pair terms, with every lane of the wave (a lane
        // that does not walk has no pieces), so that the wave can share out
        // its pair terms where contacts are many and uneven: batched (dense
        // simulations), the 4-wide walk (clustered agents) and, with SHARE,
        // the 2-wide walk of one simulation (agents with several contacts)
        if (!walks) P.mask = 0u;
        ForceSum acc;
        uint32_t tcnt = 0;   // contacts taped (TAPE; a full build: canonical slot u - n)
        auto tape = [&](uint32_t k) {
            if constexpr (TAPE) {
                for (uint32_t r = 0; r < k; ++r) {
                    const uint32_t uj = L.queue[r * bs + threadIdx.x];
                    if (uj < n) raise_error(b.g, kErrInternal);
                    if (append && tcnt < kTapeWidth) a.tape.list[size_t(tcnt) * n + (u - n)] = uj - n;
                    ++tcnt;
                }
            }
        };
        force_of<CH, T, false, BATCHED || CH == 4 || SHARE>(b, *Gp, p, P, L, acc, tape);
        if constexpr (TAPE) {
            if (inc) raise_error(b.g, kErrInternal);
            // a grid that overflowed leaves the tape incomplete
            if (active && !Gp->valid) tcnt = 0xFFFFFFFFu;
            if (active && append && Gp->valid) {
                a.tape.cnt[u - n] = tcnt;
                // with a re-layout the grid build wrote the next state's ids
                // in canonical order; else the storage index gives the id
                a.tape.ids[u - n] = RELAYOUT ? b.ids[a.ids_cur ^ 1][u - n] : b.ids[a.ids_cur][i];
                static_cast<V4<T>*>(a.tape.pos)[u - n] = p;
            }
            uint32_t most = tcnt;   // one atomic per wave
            for (int d = 32; d >= 1; d >>= 1) most = max(most, uint32_t(__shfl_xor(int(most), d, 64)));
            if (lane_id() == 0 && most > 0) atomicMax(a.tape.worst, most);
        }
        // ---- after the walk, per agent
        if (active && Gp->valid) {
            const SimGrid& G = *Gp;
            if (walks) is_static = cand && !acc.moved_near;
            V4<T> np = p;
            uint32_t nf = 0;
            if (is_static) {
                nf = kStaticBit | (f & ~(kMovedBit | kStaticBit | kBoxChangedBit));
            } else {
                const Move m = displacement(G, acc.fx, acc.fy, acc.fz);
                np.x = T(double(p.x) + m.ux);
                np.y = T(double(p.y) + m.uy);
                np.z = T(double(p.z) + m.uz);
                moved = m.ux != 0.0 || m.uy != 0.0 || m.uz != 0.0;
                st_f[0] = acc.fx;
                st_f[1] = acc.fy;
                st_f[2] = acc.fz;
                st_d = (unsigned long long)__double_as_longlong(m.size);
                const uint32_t nz = acc.nnz < 0xFFFFFFu ? acc.nnz : 0xFFFFFFu;
                nf = (moved ? kMovedBit : 0u) | (nz << kNnzShift);
                if (moved) np.w = -np.w;
                if (KEEP_F) {
                    b.force[nxt][3 * size_t(out)] = acc.fx;
                    b.force[nxt][3 * size_t(out) + 1] = acc.fy;
                    b.force[nxt][3 * size_t(out) + 2] = acc.fz;
                }
            }
            pout[out] = np;
            ok = box_coord(double(np.x), G.inv_h, &cnew[0]) && box_coord(double(np.y), G.inv_h, &cnew[1]) &&
                 box_coord(double(np.z), G.inv_h, &cnew[2]);
            // left the box it was ranked in (the next grid build re-ranks it);
            // that box is recomputed from p, so q need not live through the walk
            int32_t cold[3];
            bool left = !ok || !(box_coord(double(p.x), G.inv_h, &cold[0]) && box_coord(double(p.y), G.inv_h, &cold[1]) &&
                                 box_coord(double(p.z), G.inv_h, &cold[2]));
            for (int c = 0; c < 3; ++c) left = left || cnew[c] != cold[c];
            b.flags[nxt][out] = nf | (left ? kBoxChangedBit : 0u);
        }
        if (active && !ok) raise_error(b.g, kErrNonfinite);
        // ---- box extent and statistics: wave, then block (LDS atomics)
        const bool contrib = active && ok;
        const unsigned long long any = __ballot(contrib);
        const uint32_t ns = uint32_t(__popcll(__ballot(active && is_static)));
        const uint32_t nm = uint32_t(__popcll(__ballot(active && moved)));
        const int lead = any ? __ffsll((long long)any) - 1 : 0;
        const int wsim = __shfl(sim, lead, 64);
        const bool uniform = __ballot(contrib && sim != wsim) == 0;
        if (uniform) {
            int32_t lo[3], hi[3];
            for (int c = 0; c < 3; ++c) {
                lo[c] = wave_min(contrib ? cnew[c] : INT32_MAX);
                hi[c] = wave_max(contrib ? cnew[c] : INT32_MIN);
            }
            const int slot = wsim - sim0;
            if (lane_id() == 0 && any) {
                if (slot >= 0 && slot < kMaxBlockSims) {
                    s_sims[slot] = wsim;
                    for (int c = 0; c < 3; ++c) {
                        atomicMin(&s_box[slot][c], lo[c]);
                        atomicMax(&s_box[slot][3 + c], hi[c]);
                    }
                } else {
                    bbox_atomic(bbox_replica(b, a.parity ^ 1, wsim), lo, hi);
                }
            }
        } else if (contrib) {
            // several simulations in one wave (batched, small simulations)
            bbox_atomic(bbox_replica(b, a.parity ^ 1, sim), cnew, cnew);
        }
        if (lane_id() == 0) {
            if (ns) atomicAdd(&s_cnt[0], ns);
            if (nm) atomicAdd(&s_cnt[1], nm);
        }
        // the sum of the evaluated forces and the largest displacement: a
        // butterfly over the wave (a fixed order), into the wave's LDS slot;
        // a wave of static agents has nothing to add
        if (__ballot(active && !is_static && ok) != 0ull) {
            for (int d = 32; d >= 1; d >>= 1) {
                for (int c = 0; c < 3; ++c) st_f[c] += __shfl_xor(st_f[c], d, 64);
                const unsigned long long o = __shfl_xor(st_d, d, 64);
                st_d = o > st_d ? o : st_d;
            }
            if (lane_id() == 0) {
                const int w = int(threadIdx.x >> 6);
                for (int c = 0; c < 3; ++c) s_fsum[w][c] += st_f[c];
                s_dmax[w] = st_d > s_dmax[w] ? st_d : s_dmax[w];
            }
        }
    };
    if constexpr (two_chunks<CH>()) {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 0 && has_a) chunk_agents(n + ka * bs, true);
            if (pass == 1 && has_s) chunk_agents(ks * bs, false);
        }
    } else {
        chunk_agents(has_a ? n + ka * bs : ks * bs, has_a);
    }
    // ---- the last wave of the block to finish adds the block's result to the replicas
    if (lane_id() == 0) {
        __threadfence_block();
        const uint32_t nwaves = (blockDim.x + 63u) >> 6;
        if (atomicAdd(&s_cnt[2], 1u) == nwaves - 1) {
            __threadfence_block();
            // the waves' force sums in wave order, their largest displacement
            // (the other waves' LDS writes precede their counter increments)
            double fs[3] = {0.0, 0.0, 0.0};
            unsigned long long dm = 0ull;
            for (uint32_t w = 0; w < nwaves; ++w) {
                for (int c = 0; c < 3; ++c) fs[c] += s_fsum[w][c];
                const unsigned long long x = s_dmax[w];
                dm = x > dm ? x : dm;
            }
            if constexpr (!BATCHED) {
                // one simulation: the block's record, folded by k_fold_parts
                BlockPart r;
                for (int c = 0; c < 6; ++c) r.box[c] = atomicAdd(&s_box[0][c], 0);
                r.n_static = atomicAdd(&s_cnt[0], 0u);
                r.n_moved = atomicAdd(&s_cnt[1], 0u);
                for (int c = 0; c < 3; ++c) r.fsum[c] = fs[c];
                r.dmax = dm;
                b.bpart[blockIdx.x] = r;
                return;
            }
            {   // batched: straight to the replicas (the order of the sums is not fixed)
                const uint32_t rep = blockIdx.x % kReplicas;
                for (int c = 0; c < 3; ++c)
                    if (fs[c] != 0.0) atomicAdd(&b.g->fsum[a.parity][rep][c], fs[c]);
                if (dm) atomicMax(&b.g->dmax[a.parity][rep], dm);
            }
            for (int k = 0; k < kMaxBlockSims; ++k) {
                const int sk = atomicAdd(&s_sims[k], 0);
                if (sk < 0) continue;
                int32_t lo[3], hi[3];
                for (int c = 0; c < 3; ++c) {
                    lo[c] = atomicAdd(&s_box[k][c], 0);
                    hi[c] = atomicAdd(&s_box[k][3 + c], 0);
                }
                bbox_atomic(bbox_replica(b, a.parity ^ 1, sk), lo, hi);
            }
            const uint32_t ts = atomicAdd(&s_cnt[0], 0u), tm = atomicAdd(&s_cnt[1], 0u);
            unsigned long long* st = b.g->stats[a.parity][blockIdx.x % kReplicas];
            if (ts) atomicAdd(&st[0], (unsigned long long)ts);
            if (tm) atomicAdd(&st[1], (unsigned long long)tm);
        }
    }
}

// The step kernel's block records (one simulation) folded into replica r =
// blockIdx.x of the box-extent accumulators (slot `slot`) and of the step
// statistics (parity `parity`): each replica has one writer, so plain
// stores replace the same-address atomics of one set per block.  Block r
// folds records [r * per, (r + 1) * per).
constexpr int kFoldThreads = 256;
__global__ __launch_bounds__(kFoldThreads) void k_fold_parts(const BlockPart* __restrict__ parts, uint32_t nparts,
                                                             int32_t* __restrict__ rep, Globals* g, int slot,
                                                             int parity) {
    __shared__ int32_t s_box[kFoldThreads / 64][6];
    __shared__ unsigned long long s_cnt[kFoldThreads / 64][3];
    __shared__ double s_fs[kFoldThreads / 64][3];
    const uint32_t per = (nparts + kReplicas - 1) / kReplicas;
    const uint32_t e0 = blockIdx.x * per, e1 = min(e0 + per, nparts);
    int32_t box[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
    unsigned long long cnt[3] = {0ull, 0ull, 0ull};   // static, moved, largest displacement
    double fs[3] = {0.0, 0.0, 0.0};
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kFoldThreads) {   // each thread in record order
        const BlockPart r = parts[e];
        for (int a = 0; a < 3; ++a) {
            box[a] = min(box[a], r.box[a]);
            box[3 + a] = max(box[3 + a], r.box[3 + a]);
            fs[a] += r.fsum[a];
        }
        cnt[0] += r.n_static;
        cnt[1] += r.n_moved;
        cnt[2] = r.dmax > cnt[2] ? r.dmax : cnt[2];
    }
    const int wave = int(threadIdx.x >> 6);
    for (int a = 0; a < 3; ++a) {
        box[a] = wave_min(box[a]);
        box[3 + a] = wave_max(box[3 + a]);
    }
    for (int d = 32; d >= 1; d >>= 1) {   // a fixed order: the sums do not depend on timing
        for (int c = 0; c < 2; ++c) cnt[c] += __shfl_xor(cnt[c], d, 64);
        const unsigned long long o = __shfl_xor(cnt[2], d, 64);
        cnt[2] = o > cnt[2] ? o : cnt[2];
        for (int c = 0; c < 3; ++c) fs[c] += __shfl_xor(fs[c], d, 64);
    }
    if (lane_id() == 0) {
        for (int a = 0; a < 6; ++a) s_box[wave][a] = box[a];
        for (int c = 0; c < 3; ++c) {
            s_cnt[wave][c] = cnt[c];
            s_fs[wave][c] = fs[c];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFoldThreads / 64; ++w) {
            for (int a = 0; a < 3; ++a) {
                box[a] = min(box[a], s_box[w][a]);
                box[3 + a] = max(box[3 + a], s_box[w][3 + a]);
                fs[a] += s_fs[w][a];
            }
            cnt[0] += s_cnt[w][0];
            cnt[1] += s_cnt[w][1];
            cnt[2] = s_cnt[w][2] > cnt[2] ? s_cnt[w][2] : cnt[2];
        }
        int32_t* t = rep + (size_t(slot) * kReplicas + blockIdx.x) * 6;   // one simulation
        for (int a = 0; a < 6; ++a) t[a] = box[a];
        g->stats[parity][blockIdx.x][0] = cnt[0];
        g->stats[parity][blockIdx.x][1] = cnt[1];
        for (int c = 0; c < 3; ++c) g->fsum[parity][blockIdx.x][c] = fs[c];
        g->dmax[parity][blockIdx.x] = cnt[2];
    }
}

uint32_t force_part_capacity(uint32_t n) { return 2u * ((n + 63u) / 64u) + 1024u; }

template <class T>
void launch_fold_parts(const Buffers<T>& b, uint32_t nparts, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_parts, dim3(kReplicas), dim3(kFoldThreads), 0, s, b.bpart, nparts, b.bbox_rep, b.g,
                       parity ^ 1, parity);
}

template <class T, bool S, bool K, bool R, int CH, bool TAPE = false, bool SH = false>
static void launch_force_v(const Buffers<T>& b, const StepArgs& a, hipStream_t s) {
    const int bs = a.block_size;
    const uint32_t nb = (b.n + bs - 1) / bs;
    // two chunks per block; or one, and storage chunks hold agents only in
    // an update build
    const uint32_t first = two_chunks<CH>() || !a.full_only ? 0u : nb;
    const uint32_t blocks = two_chunks<CH>() ? nb : 2u * nb - first;
    const uint32_t run = xcd_run(blocks);
    const uint32_t grid = xcd_grid(blocks, run);   // <= force_part_capacity(n): nb <= ceil(n / 64), 8 run <= 512
    hipLaunchKernelGGL((k_force<T, S, K, R, CH, TAPE, SH>), dim3(grid), dim3(bs), walk_lds_bytes<CH>(bs), s, b, a, run,
                       first);
    if (!S) launch_fold_parts(b, grid, a.parity, s);
}

// the shared pair terms of the 2-wide walk of one simulation are a variant of
// their own (the 4-wide walk and a batch always share)
template <class T, bool S, bool K, bool R, int CH, bool TAPE = false>
static void launch_force_s(const Buffers<T>& b, const StepArgs& a, hipStream_t s) {
    if constexpr (CH == 2 && !S) {
        if (a.share) {
            launch_force_v<T, S, K, R, CH, TAPE, true>(b, a, s);
            return;
        }
    }
    launch_force_v<T, S, K, R, CH, TAPE>(b, a, s);
}

template <class T, int CH>
static void launch_force_c(const Buffers<T>& b, const StepArgs& a, hipStream_t s) {
    const int v = (b.sim_of ? 4 : 0) | (a.detect_static ? 2 : 0) | (a.relayout ? 1 : 0);
    if (a.tape.pos && v <= 1) {   // the host tapes no other kind of step
        if (v == 1)
            launch_force_s<T, false, false, true, CH, true>(b, a, s);
        else
            launch_force_s<T, false, false, false, CH, true>(b, a, s);
        return;
    }
    switch (v) {
        case 0: launch_force_s<T, false, false, false, CH>(b, a, s); break;
        case 1: launch_force_s<T, false, false, true, CH>(b, a, s); break;
        case 2: launch_force_s<T, false, true, false, CH>(b, a, s); break;
        case 3: launch_force_s<T, false, true, true, CH>(b, a, s); break;
        case 4: launch_force_s<T, true, false, false, CH>(b, a, s); break;
        case 5: launch_force_s<T, true, false, true, CH>(b, a, s); break;
        case 6: launch_force_s<T, true, true, false, CH>(b, a, s); break;
        default: launch_force_s<T, true, true, true, CH>(b, a, s); break;
    }
}

template <class T>
void launch_force(const Buffers<T>& b, const StepArgs& a, hipStream_t s) {
    if (a.walk_chunk == 4)
        launch_force_c<T, 4>(b, a, s);
    else
        launch_force_c<T, 2>(b, a, s);
}

// ------------------------------------------------------------------ neighbour sets
// N(i) of every agent on the positions of the last grid (a query, not part of
// the step): the walk of the step, the exact test |e|^2 < R^2 in double.
// rows == nullptr: counts[id] = |N(i)|.  Otherwise row id of `rows` (width
// K) gets the neighbour ids in ascending order (insertion), and *worst the
// largest count.  One thread per loose slot of the grid.
template <class T>
__device__ __forceinline__ uint32_t loose_storage(const Buffers<T>& b, uint32_t u) {
    return u < b.n ? u : b.perm[u - b.n];
}

template <class T>
__global__ __launch_bounds__(256) void k_neighbors(Buffers<T> b, int ids_cur, uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ rows, uint32_t K, uint32_t* worst) {
    extern __shared__ __align__(16) unsigned char s_walk[];
    const WalkLds L = walk_lds(s_walk);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2u * b.n) return;
    const bool live = t < b.n ? (b.g->inc && b.gkey[t] != kDeadKey) : t - b.n < min(b.g->napp, b.n);
    if (!live) return;
    const uint32_t* ids = b.ids[ids_cur];
    const uint32_t i = loose_storage(b, t);
    const uint32_t id = i < b.n ? ids[i] : 0xFFFFFFFFu;
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const SimGrid& G = b.sims[sim_index(b, i)];
    const V4<T> p = gpos_ptr(b)[t];
    uint32_t q[3];
    if (!G.valid || !box_of<T>(G, p, q)) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const Pieces P = load_pieces(b, G, q, G.stamp, L);
    const double xi = double(p.x), yi = double(p.y), zi = double(p.z);
    uint32_t cnt = 0;
    uint32_t* row = rows ? rows + size_t(id) * K : nullptr;
    stream_pieces(L, P, [&](uint32_t u) {
        if (u == t) return true;
        const V4<T> pj = gpos_ptr(b)[u];
        const double ex = xi - double(pj.x), ey = yi - double(pj.y), ez = zi - double(pj.z);
        if (!(((ex * ex + ey * ey) + ez * ez) < G.r2)) return true;
        if (row && cnt < K) {
            const uint32_t j = loose_storage(b, u);
            const uint32_t jd = j < b.n ? ids[j] : 0xFFFFFFFFu;
            uint32_t x = cnt;
            while (x > 0 && row[x - 1] > jd) {
                row[x] = row[x - 1];
                --x;
            }
            row[x] = jd;
        }
        ++cnt;
        return true;
    });
    if (row)
        for (uint32_t x = cnt; x < K; ++x) row[x] = 0xFFFFFFFFu;
    else
        counts[id] = cnt;
    if (worst) atomicMax(worst, cnt);
}

template <class T>
void launch_neighbors(const Buffers<T>& b, int ids_cur, uint32_t* counts, uint32_t* rows, uint32_t K,
                      uint32_t* worst, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors<T>, dim3((2u * b.n + 255) / 256), dim3(256), walk_lds_bytes<4>(256), s, b, ids_cur,
                       counts, rows, K, worst);
}

// ------------------------------------------------------------------ copies
template <class T>
__global__ void k_unpack_positions(Buffers<T> b, int cur, int ids_cur, T* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const uint32_t id = b.ids[ids_cur][i];
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const V4<T> p = pos4_ptr(b, cur)[i];
    out[3 * size_t(id)] = p.x;
    out[3 * size_t(id) + 1] = p.y;
    out[3 * size_t(id) + 2] = p.z;
}

template <class T>
void launch_unpack_positions(const Buffers<T>& b, int pos_cur, int ids_cur, T* out, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack_positions<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, pos_cur, ids_cur, out);
}

// field: 1 forces, 2 moved, 3 static, 4 nnz, 9 storage ids
template <class T>
__global__ void k_unpack_field(Buffers<T> b, int cur, int ids_cur, int field, void* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const uint32_t* ids = b.ids[ids_cur];
    if (field == 9) {
        static_cast<uint32_t*>(out)[i] = ids[i];
        return;
    }
    const uint32_t id = ids[i];
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    const uint32_t f = b.flags[cur][i];
    switch (field) {
        case 1:
            for (int c = 0; c < 3; ++c) static_cast<double*>(out)[3 * size_t(id) + c] = b.force[cur][3 * size_t(i) + c];
            break;
        case 2: static_cast<uint8_t*>(out)[id] = uint8_t(f & kMovedBit); break;
        case 3: static_cast<uint8_t*>(out)[id] = uint8_t((f & kStaticBit) ? 1 : 0); break;
        case 4: static_cast<int32_t*>(out)[id] = int32_t(f >> kNnzShift); break;
        case 12: static_cast<T*>(out)[id] = T(fabs(double(pos4_ptr(b, cur)[i].w))); break;
        default: break;
    }
}

template <class T>
void launch_unpack_field(const Buffers<T>& b, int pos_cur, int ids_cur, int field, void* out, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack_field<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, pos_cur, ids_cur, field, out);
}

template <class T>
__global__ void k_load_positions(Buffers<T> b, int cur, int ids_cur, const T* __restrict__ in) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const uint32_t id = b.ids[ids_cur][i];
    if (id >= b.n) {
        raise_error(b.g, kErrInternal);
        return;
    }
    V4<T>* p = pos4_ptr(b, cur);
    V4<T> v = p[i];
    v.x = in[3 * size_t(id)];
    v.y = in[3 * size_t(id) + 1];
    v.z = in[3 * size_t(id) + 2];
    if (!isfinite(double(v.x)) || !isfinite(double(v.y)) || !isfinite(double(v.z))) raise_error(b.g, kErrNonfinite);
    p[i] = v;
}

template <class T>
void launch_load_positions(const Buffers<T>& b, int pos_cur, int ids_cur, const T* in, hipStream_t s) {
    hipLaunchKernelGGL(k_load_positions<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, pos_cur, ids_cur, in);
}

// moved / nnz given by id (import of a checkpoint); storage slot i holds id ids[i]
template <class T>
__global__ void k_set_flags(Buffers<T> b, int cur, const uint8_t* __restrict__ moved,
                            const int32_t* __restrict__ nnz, const uint32_t* __restrict__ ids) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n) return;
    const uint32_t id = ids[i];
    if (id >= b.n) return;
    const uint32_t nz = uint32_t(max(nnz[id], 0));
    b.flags[cur][i] = (moved[id] ? kMovedBit : 0u) | ((nz < 0xFFFFFFu ? nz : 0xFFFFFFu) << kNnzShift);
}

template <class T>
void launch_set_flags(const Buffers<T>& b, int pos_cur, int ids_cur, const uint8_t* moved, const int32_t* nnz,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_set_flags<T>, dim3((b.n + 255) / 256), dim3(256), 0, s, b, pos_cur, moved, nnz,
                       static_cast<const uint32_t*>(b.ids[ids_cur]));
}

#define ABM_INSTANTIATE(T)                                                                                   \
    template void launch_force<T>(const Buffers<T>&, const StepArgs&, hipStream_t);                        \
    template void launch_fold_parts<T>(const Buffers<T>&, uint32_t, int, hipStream_t);                     \
    template void launch_neighbors<T>(const Buffers<T>&, int, uint32_t*, uint32_t*, uint32_t, uint32_t*,   \
                                      hipStream_t);                                                         \
    template void launch_unpack_positions<T>(const Buffers<T>&, int, int, T*, hipStream_t);                \
    template void launch_unpack_field<T>(const Buffers<T>&, int, int, int, void*, hipStream_t);            \
    template void launch_load_positions<T>(const Buffers<T>&, int, int, const T*, hipStream_t);            \
    template void launch_set_flags<T>(const Buffers<T>&, int, int, const uint8_t*, const int32_t*, hipStream_t);

ABM_INSTANTIATE(float)
ABM_INSTANTIATE(double)

}  // namespace abm
