// Per-mode sparse MTTKRP (optionally with the dynamic remap in the same
// pass), the residual (loss-gradient) variant and the sampled-loss forward,
// which share one kernel template, and the standalone remap, templated on
// the number of modes N and the factor storage type.
//
// Work decomposition.  The tensor buffer holds layout L_n: nonzeros
// contiguous by output row c_n (Sec. III-B).  The plan cuts it into shards
// of at most g nonzeros that never cross a super-shard (Sec. III-A); one
// wave64 processes one shard.  Lanes run along the rank: a nonzero is
// handled by LANES lanes holding V consecutive ranks each (16 or 32 bytes
// of factor row per lane), so one step covers SW = 64/LANES nonzeros, one
// per lane group ("slot"); the shard is cut into SW contiguous runs, one per
// slot.
//
// Per nonzero (elementwise update, Sec. II-C / Eq. 4): gather the N-1 input
// factor rows, form their Hadamard product in registers, scale by the
// value.  Rows that start and end inside a slot's run are accumulated in
// registers and written at once; the runs' first and last rows are joined
// by one segmented scan over the slots, so every output row is produced by
// one wave in a fixed order.  The shard's first row (if it began in an
// earlier shard) and last row (if it continues) go to a per-shard partial
// slot that the carry fix-up kernel adds in shard order.  No global atomics
// anywhere (lock-free ownership of output rows, Sec. IV).
//
// Remap (Alg. "Dynasor", store into the next mode's shard): by default a
// separate kernel right after the MTTKRP (remap_kernel, below); with the
// FUSE form, lane 0 of each slot copies the whole record to L_{n+1}[P_n[e]],
// the slot precomputed by the plan, in the MTTKRP pass itself (the paper's
// same-agent form, Sec. V-B).
#pragma once
#include "common.hpp"
#include "launch.hpp"

namespace mk {



// ---- lane rank sets -------------------------------------------------------
// Contiguous: lane `sub` owns ranks [sub*V, sub*V + V); needs R % V == 0 and
// 16-byte aligned rows.  Strided (any R): lane `sub` of 64 owns ranks
// sub + 64*j, j < V.
template <typename FT, int V, bool STRIDED>
struct Fetch;

template <>
struct Fetch<float, 4, false> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[4])
    {
        const float4 v = *reinterpret_cast<const float4 *>(
            reinterpret_cast<const float *>(A) + row * R + sub * 4);
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    }
};

template <>
struct Fetch<float, 8, false> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[8])
    {
        const float4 *q = reinterpret_cast<const float4 *>(
            reinterpret_cast<const float *>(A) + row * R + sub * 8);
        const float4 v0 = q[0], v1 = q[1];
        x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
        x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
    }
};

template <>
struct Fetch<uint16_t, 16, false> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[16])
    {
        const uint4 *q = reinterpret_cast<const uint4 *>(
            reinterpret_cast<const uint16_t *>(A) + row * R + sub * 16);
        const uint4 u0 = q[0], u1 = q[1];
        x[0] = bf16lo(u0.x); x[1] = bf16hi(u0.x); x[2] = bf16lo(u0.y); x[3] = bf16hi(u0.y);
        x[4] = bf16lo(u0.z); x[5] = bf16hi(u0.z); x[6] = bf16lo(u0.w); x[7] = bf16hi(u0.w);
        x[8] = bf16lo(u1.x); x[9] = bf16hi(u1.x); x[10] = bf16lo(u1.y); x[11] = bf16hi(u1.y);
        x[12] = bf16lo(u1.z); x[13] = bf16hi(u1.z); x[14] = bf16lo(u1.w); x[15] = bf16hi(u1.w);
    }
};

template <>
struct Fetch<uint16_t, 8, false> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[8])
    {
        const uint4 u = *reinterpret_cast<const uint4 *>(
            reinterpret_cast<const uint16_t *>(A) + row * R + sub * 8);
        x[0] = bf16lo(u.x); x[1] = bf16hi(u.x);
        x[2] = bf16lo(u.y); x[3] = bf16hi(u.y);
        x[4] = bf16lo(u.z); x[5] = bf16hi(u.z);
        x[6] = bf16lo(u.w); x[7] = bf16hi(u.w);
    }
};

template <int V>
struct Fetch<float, V, true> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[V])
    {
        const float *p = reinterpret_cast<const float *>(A) + row * R;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int r = sub + 64 * j;
            const float v = p[r < R ? r : R - 1];     // clamped: no branch
            x[j] = (r < R) ? v : 0.0f;
        }
    }
};

template <int V>
struct Fetch<uint16_t, V, true> {
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               float (&x)[V])
    {
        const uint16_t *p = reinterpret_cast<const uint16_t *>(A) + row * R;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int r = sub + 64 * j;
            const float v = bf16_to_f32(p[r < R ? r : R - 1]);
            x[j] = (r < R) ? v : 0.0f;
        }
    }
};

template <int V, bool STRIDED>
__device__ __forceinline__ void store_row(float *dst, int R, int sub, const float (&v)[V])
{
    if constexpr (STRIDED) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            int r = sub + 64 * j;
            if (r < R) dst[r] = v[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; j += 4)
            *reinterpret_cast<float4 *>(dst + sub * V + j) =
                make_float4(v[j], v[j + 1], v[j + 2], v[j + 3]);
    }
}

template <int LANES, int V, bool STRIDED>
__device__ __forceinline__ bool lane_active(int sub, int R)
{
    if constexpr (STRIDED) return sub < R;
    else return sub * V < R;
}

// A lane's piece of a factor row as raw 32-bit words (contiguous lane forms):
// RW = V * sizeof(FT) / 4 words, loaded as 16-byte vectors, and its
// conversion to V floats (FP32: the words themselves; BF16: two values per
// word, low half first, as in Fetch).
template <typename FT, int V>
struct RawRow {
    static constexpr int RW = V * (int)sizeof(FT) / 4;
    static_assert(RW % 4 == 0, "whole 16-byte vectors");
    static __device__ __forceinline__ void get(const void *A, int64_t row, int R, int sub,
                                               uint32_t (&w)[RW])
    {
        const uint4 *q = reinterpret_cast<const uint4 *>(
            reinterpret_cast<const FT *>(A) + row * R + sub * V);
#pragma unroll
        for (int i = 0; i < RW / 4; ++i) {
            const uint4 u = q[i];
            w[4 * i] = u.x; w[4 * i + 1] = u.y; w[4 * i + 2] = u.z; w[4 * i + 3] = u.w;
        }
    }
    static __device__ __forceinline__ void unpack(const uint32_t (&w)[RW], float (&x)[V])
    {
        if constexpr (sizeof(FT) == 4) {
#pragma unroll
            for (int j = 0; j < V; ++j) x[j] = __uint_as_float(w[j]);
        } else {
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                x[2 * i] = bf16lo(w[i]);
                x[2 * i + 1] = bf16hi(w[i]);
            }
        }
    }
};

// The N-1 input modes of output mode n in the layout's key order
// n-1, n-2, ..., n+1 (cyclic, uniform).  Input 0 is the layout's second
// key: inside an output row the nonzeros are sorted by it.
template <int N>
struct Inputs {
    const void *fac[N > 1 ? N - 1 : 1];
    uint32_t off[N > 1 ? N - 1 : 1], msk[N > 1 ? N - 1 : 1];   // coordinate in a record
    __device__ __forceinline__ Inputs(const Args &a, int n)
    {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            const int w = (n + N - 1 - k) % N;
            fac[k] = a.fac[w];
            off[k] = a.coff[w];
            msk[k] = a.cmask[w];
        }
    }
};

// Product of the factor rows of inputs K0..N-2 of one nonzero (ones when
// there are none).  Every load is unconditional (the caller passes an
// in-range record and lane), so the compiler can keep all gathers of an
// unrolled group in flight at once.
template <int N, int W, typename FT, int V, bool STRIDED, int K0>
__device__ __forceinline__ void row_product(const Inputs<N> &in, const Rec<W> &rc, int R,
                                            int sub, float (&pr)[V])
{
#pragma unroll
    for (int j = 0; j < V; ++j) pr[j] = 1.0f;
#pragma unroll
    for (int k = K0; k < N - 1; ++k) {
        float x[V];
        Fetch<FT, V, STRIDED>::get(in.fac[k], (int64_t)rec_coord<W>(rc, in.off[k], in.msk[k]), R,
                                   sub, x);
#pragma unroll
        for (int j = 0; j < V; ++j) pr[j] *= x[j];
    }
}

// Sum over the LANES lanes of one slot (xor butterfly stays inside the slot).
template <int LANES>
__device__ __forceinline__ float slot_sum(float v)
{
#pragma unroll
    for (int m = LANES / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// ---- per-mode MTTKRP family ---------------------------------------------
// KIND (a Kind of launch.hpp):
//   KIND_MTTKRP  M_n(i,:) = sum_e v_e * prod_{w != n} A_w(c_w(e), :)
//   KIND_RESID   loss-gradient pass: the same sum with v_e replaced by
//                -2 s rho_e, rho_e = v_e - m_e recomputed from the model
//                value m_e = sum_r A_n(c_n(e), r) prod_{w != n} A_w(c_w(e), r)
//   KIND_LOSS    loss forward: sum_e rho_e^2, one FP64 partial per shard
//                (FP32 terms, FP64 accumulation); no output rows
//   KIND_RESID_LOSS  KIND_RESID that also writes KIND_LOSS's partials (the
//                same terms in the same order), so a loss-and-gradient
//                evaluation needs no separate loss pass
//   KIND_GATHER  measurement only: the same record loads, factor-row
//                gathers, row reuse and products, but every product is added
//                into one register per lane and stored to the shard's first
//                output row, with no segmentation; its time is the cost of
//                the loads themselves, a ceiling for this kernel
//
// The wave's shard is cut into SW equal contiguous runs, one per slot.  A
// slot walks its run in order, U nonzeros per iteration (all their loads
// issued before the first use), accumulating the current row in registers:
// a row that starts and ends inside the run is complete and written at
// once.  The first row of each run (head) and the last (tail) are then
// joined across slots with one segmented scan per shard.
template <int N, int W, typename FT, int LANES, int V, bool STRIDED, int KIND, bool FUSE>
__global__ __launch_bounds__(MTT_WAVES * 64) void mttkrp_kernel(Args a)
{
    constexpr bool RLOSS = KIND == KIND_RESID_LOSS;
    constexpr bool RESID = KIND == KIND_RESID || RLOSS;
    constexpr bool LOSS = KIND == KIND_LOSS;
    constexpr bool GONLY = KIND == KIND_GATHER;
    constexpr bool MODEL = RESID || LOSS;        // m_e needed: output row gathered too
    constexpr int SW = WAVE / LANES;
    // nonzeros per step of a lane group: 4 measured fastest (2 and 3 keep
    // fewer gathers in flight; 8 halves the waves per SIMD and is slower)
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const int sidx = blockIdx.x * MTT_WAVES + (threadIdx.x >> 6);
    if (sidx >= a.nshards) return;                         // whole wave
    const int shard = a.order ? a.order[sidx] : sidx;
    const int start = a.shards[3 * shard];
    const int len = a.shards[3 * shard + 1];
    const int end = start + len;
    const int n = a.mode, R = a.R;
    const int slot = lane / LANES, sub = lane % LANES;
    const bool ract = lane_active<LANES, V, STRIDED>(sub, R);
    // the shard's first and last output rows (plan table); records do not
    // store c_n, which the row-start table of L_n recovers per position
    const int f = a.fl[2 * shard], l = a.fl[2 * shard + 1];
    const bool split_before = a.row_ptr[f] < start;
    float coef = 1.0f;
    if constexpr (RESID) coef = -2.0f * (a.gscale ? (float)a.gscale[0] : 1.0f);
    float *const cbase = a.carry + (int64_t)shard * 2 * R;

    float *const out = a.out;
    // a complete row, or the shard's first row when it began earlier
#define FLUSH_MID(row, v)                                                            \
    store_row<V, STRIDED>(((row) == f && split_before) ? cbase : out + (int64_t)(row) * R, \
                          R, sub, v)

    const int run = (len + SW - 1) / SW;
    const int s0 = start + slot * run;
    const int s1 = min(s0 + run, end);           // s0 >= s1: empty run (row l)
    float acc[V], head[V];
#pragma unroll
    for (int j = 0; j < V; ++j) { acc[j] = 0.0f; head[j] = 0.0f; }

    const Inputs<N> in(a, n);
    const int fsub = ract ? sub : 0;             // in-range lane for loads
    // Row reuse for the first NR inputs (contiguous lane forms).  Inside an
    // output row the nonzeros are sorted by the input-0 coordinate, then
    // input 1, so consecutive nonzeros of a slot often need the same input-0
    // row (70-99% of them on Zipf-skewed tensors) and, with five or more
    // modes, the same input-1 row (30-75%).  Such a row is loaded only when
    // its coordinate changes and the slot uses the row it loaded last; the
    // products are the same.  NR = 1, or 2 from five modes on, and from
    // four modes on with BF16 factors (measured; with four modes and FP32
    // factors the registers of a second input cost more occupancy than the
    // loads save).  The kept rows are held as the raw words loaded
    // and widened after the selection: a BF16 row then costs half the
    // registers of an FP32 one, and no conversion waits inside the
    // conditional load (widening there serialised the loads).
    constexpr int NR0 = (N >= 5 || (N == 4 && sizeof(FT) == 2)) ? 2 : 1;
    constexpr int NR = (!STRIDED && N > 2) ? (N - 2 < NR0 ? N - 2 : NR0) : 0;
    constexpr bool REUSE = NR > 0;
    constexpr int RW = STRIDED ? 1 : V * (int)sizeof(FT) / 4;
    uint32_t xp[NR > 0 ? NR : 1][RW];
    int pc[NR > 0 ? NR : 1];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        pc[k] = -1;
#pragma unroll
        for (int j = 0; j < RW; ++j) xp[k][j] = 0u;
    }
    // Records are loaded once per lane group, not once per lane: lane `sub`
    // of a slot loads records sub, sub + LANES, ... of the slot's next U
    // nonzeros (RPL per lane), and the words are then broadcast inside the
    // slot with cross-lane moves.  The vector-memory path (misses in flight
    // per CU) limits this kernel, so duplicate loads are expensive.  The
    // next group's records are loaded while the current group computes.
    // The loss kinds also need the output-mode row of every nonzero for the
    // model value.  It is constant along a run of one output row (about
    // nnz / I_n nonzeros), so it is likewise loaded only when the row changes
    // (contiguous lane forms).
    constexpr bool OREUSE = MODEL && !STRIDED;
    uint32_t xo[RW];
    int po = -1;
#pragma unroll
    for (int j = 0; j < RW; ++j) xo[j] = 0u;
    double lacc = 0.0;                            // KIND_LOSS: sum of rho^2
    constexpr int RPL = (U + LANES - 1) / LANES;
    // Output rows.  A slot's run is walked in segments of 64 positions,
    // [s0 + 64m, s0 + 64m + 64), which never split a step (64 is a multiple
    // of U) and span at most two 64-position blocks of the row-start table.
    // When the positions it loads next open a segment, the slot builds the
    // segment's 64-bit start mask from two table entries; each step then
    // takes its U start bits with one shift and keeps a running count of
    // rows started (the ordinal that indexes the list of nonempty rows).
    // Every slot of the wave opens its next segment at the same step, so
    // the mask is built under a wave-uniform branch once per 64 / U steps,
    // from entries loaded one segment earlier: segment m needs the entries
    // of blocks sblk + m and sblk + m + 1, held in ev (even offsets) and od
    // (odd offsets); the one of block sblk + m is then replaced in place by
    // that of block sblk + m + 2.  (Rotated through a third register, the
    // new entry went to a temporary whose copy waited for the load.)  The
    // row id of a position is loaded only where a row starts, and for the
    // run's first position; elsewhere nid = -1 means "the previous
    // position's row".
    constexpr int SEG = 64 / U;                  // steps per segment
    static_assert(64 % U == 0 && U <= 32, "a step never splits a 64-position segment");
    const int soff = s0 & 63, sblk = s0 >> 6;
    RowStart od = row_start_at(a.rbits, min(sblk + 1, a.nblk));
    RowStart ev = row_start_at(a.rbits, min(sblk + 2, a.nblk));
    const SegStarts sg0 = seg_starts(row_start_at(a.rbits, min(sblk, a.nblk)), od, soff);
    uint64_t smask = sg0.m;
    int orun = sg0.before;                       // rows started before the positions loaded next
    Rec<W> nxt[RPL];
    int nid[RPL];
    {
        const uint32_t bu = (uint32_t)smask & ((1u << U) - 1u);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const int u = sub + j * LANES;
            const int e = s0 + u;
            const bool v = u < U && u < run && e < end;
            nxt[j] = load_rec<W>(a.rin, v ? e : start);
            const bool st = ((bu >> (u & 31)) & 1u) != 0;
            const int o = orun + __popc(bu & ((2u << (u & 31)) - 1u)) - 1;
            nid[j] = -1;
            if (v && (st || u == 0)) nid[j] = a.nrows[max(o, 0)];   // o >= 0 when v
        }
        orun += __popc(bu);
    }
    const int r0 = __shfl(nid[0], slot * LANES);  // row of the run's first position
    int cur_row = (s0 < s1) ? r0 : l;
    const int head_row = cur_row;
    int prow = cur_row;                          // row of the previous position
    bool in_head = true;
    for (int k = 0; k < run; k += U) {           // uniform trip count
        Rec<W> rc[U];
        bool ok[U];
        int rr[U];                               // output row of each nonzero
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = s0 + k + u;
            ok[u] = (k + u < run) && (e < end);
            const int src = slot * LANES + (u % LANES);
#pragma unroll
            for (int w = 0; w < W + 1; ++w)
                rc[u].w[w] = (uint32_t)__shfl((int)nxt[u / LANES].w[w], src);
            const int id = __shfl(nid[u / LANES], src);
            rr[u] = id >= 0 ? id : (u == 0 ? prow : rr[u - 1]);
        }
        prow = rr[U - 1];
        const int q = (k + U) / U;               // step of the positions loaded next
        if (q % SEG == 0 && q * U < run) {       // they open a segment (uniform)
            const int m = q / SEG;
            int ix = min(sblk + m + 2, a.nblk);
            if (m & 1) {
                const SegStarts sg = seg_starts(od, ev, soff);
                smask = sg.m;
                orun = sg.before;
                asm volatile("" : "+v"(ix) : "v"(orun));   // load after od is read
                od = row_start_at(a.rbits, ix);
            } else {
                const SegStarts sg = seg_starts(ev, od, soff);
                smask = sg.m;
                orun = sg.before;
                asm volatile("" : "+v"(ix) : "v"(orun));   // load after ev is read
                ev = row_start_at(a.rbits, ix);
            }
        }
        const uint32_t bu = (uint32_t)(smask >> (U * (q % SEG))) & ((1u << U) - 1u);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {            // clamped index: no branch
            const int u = sub + j * LANES;
            const int e = s0 + k + U + u;
            const bool v = u < U && k + U + u < run && e < end;
            nxt[j] = load_rec<W>(a.rin, v ? e : start);
            const bool st = ((bu >> (u & 31)) & 1u) != 0;
            const int o = orun + __popc(bu & ((2u << (u & 31)) - 1u)) - 1;
            nid[j] = -1;
            if (v && st) nid[j] = a.nrows[max(o, 0)];
        }
        orun += __popc(bu);
        float pr[U][V];
        float mm[U];
        uint32_t xq[OREUSE ? U : 1][RW];
        bool ndo[U];
        if constexpr (OREUSE) {
            int co[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                co[u] = rr[u];
                ndo[u] = ok[u] && co[u] != (u == 0 ? po : co[u - 1]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int j = 0; j < RW; ++j) xq[u][j] = 0u;
                if (ndo[u]) RawRow<FT, V>::get(a.fac[n], (int64_t)co[u], R, fsub, xq[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) po = co[u];
        }
        if constexpr (REUSE) {
            int cc[NR][U];
            bool need[NR][U];
#pragma unroll
            for (int k = 0; k < NR; ++k)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    cc[k][u] = rec_coord<W>(rc[u], in.off[k], in.msk[k]);
                    need[k][u] = ok[u] && cc[k][u] != (u == 0 ? pc[k] : cc[k][u - 1]);
                }
            uint32_t xr[NR][U][RW];
#pragma unroll
            for (int k = 0; k < NR; ++k)
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int j = 0; j < RW; ++j) xr[k][u][j] = 0u;
                    if (need[k][u])
                        RawRow<FT, V>::get(in.fac[k], (int64_t)cc[k][u], R, fsub, xr[k][u]);
                }
#pragma unroll
            for (int k = 0; k < NR; ++k)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) pc[k] = cc[k][u];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                row_product<N, W, FT, V, STRIDED, NR>(in, rc[u], R, fsub, pr[u]);
#pragma unroll
                for (int k = NR - 1; k >= 0; --k) {
                    // opaque copy of the flag: keeps the compiler from
                    // folding the selection into the conditional load, which
                    // would make each load wait for the one before it
                    int sel = need[k][u] ? 1 : 0;
                    asm volatile("" : "+v"(sel));
#pragma unroll
                    for (int j = 0; j < RW; ++j) xp[k][j] = sel ? xr[k][u][j] : xp[k][j];
                    float x[V];
                    RawRow<FT, V>::unpack(xp[k], x);
#pragma unroll
                    for (int j = 0; j < V; ++j) pr[u][j] = x[j] * pr[u][j];
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                row_product<N, W, FT, V, STRIDED, 0>(in, rc[u], R, fsub, pr[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mm[u] = 0.0f;
            if constexpr (MODEL) {
                float xn[V];
                if constexpr (OREUSE) {
                    int sel = ndo[u] ? 1 : 0;        // opaque, as for the input rows
                    asm volatile("" : "+v"(sel));
#pragma unroll
                    for (int j = 0; j < RW; ++j) xo[j] = sel ? xq[u][j] : xo[j];
                    RawRow<FT, V>::unpack(xo, xn);
                } else {
                    Fetch<FT, V, STRIDED>::get(a.fac[n], (int64_t)rr[u], R, fsub, xn);
                }
#pragma unroll
                for (int j = 0; j < V; ++j) mm[u] += pr[u][j] * xn[j];
                if (!(ok[u] && ract)) mm[u] = 0.0f;
            }
        }
        if constexpr (LOSS) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // model value m_e (lanes outside the rank range hold 0)
                const float m = slot_sum<LANES>(mm[u]);
                if (ok[u] && sub == 0) {
                    const float rho = __uint_as_float(rc[u].w[W]) - m;
                    lacc += (double)(rho * rho);  // FP32 term, FP64 accumulation
                }
            }
            continue;
        }
        if constexpr (FUSE) {
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) dst[u] = a.perm[ok[u] ? s0 + k + u : start];
            const int nx = n + 1 < N ? n + 1 : 0;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u] && sub == 0)
                    store_rec<W>(a.rout, dst[u],
                                 repack<N, W>(rc[u], rr[u], n, nx, a.coff, a.ooff, a.cmask));
        }
        // the weight of each nonzero: its value, or -2 s rho for the
        // residual kinds (every lane takes part in the slot sums)
        float cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float c = 0.0f;
            if constexpr (RESID) {
                // model value m_e (lanes outside the rank range hold 0)
                const float m = slot_sum<LANES>(mm[u]);
                if (ok[u]) {
                    const float rho = __uint_as_float(rc[u].w[W]) - m;
                    c = coef * rho;
                    if constexpr (RLOSS) {
                        if (sub == 0) lacc += (double)(rho * rho);   // as KIND_LOSS
                    }
                }
            } else {
                if (ok[u]) c = __uint_as_float(rc[u].w[W]);
            }
            cv[u] = c;
        }
        if constexpr (GONLY) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) {
#pragma unroll
                    for (int j = 0; j < V; ++j) acc[j] += cv[u] * pr[u][j];
                }
            continue;
        }
        // Most steps stay inside the current row: then the products are
        // simply added.  Only a step that opens a row (or ends the run)
        // takes the per-nonzero path, which keeps the control flow and the
        // accumulator moves of row changes off the common path.
        bool same = true;
#pragma unroll
        for (int u = 0; u < U; ++u) same = same && ok[u] && rr[u] == cur_row;
        if (same) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < V; ++j) acc[j] += cv[u] * pr[u][j];
            continue;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (ok[u]) {
                const int row = rr[u];
                if (row != cur_row) {
                    if (in_head) {
#pragma unroll
                        for (int j = 0; j < V; ++j) head[j] = acc[j];
                        in_head = false;
                    } else if (ract) {
                        // interior row: starts and ends inside this run
                        store_row<V, STRIDED>(out + (int64_t)cur_row * R, R, sub, acc);
                    }
#pragma unroll
                    for (int j = 0; j < V; ++j) acc[j] = 0.0f;
                    cur_row = row;
                }
#pragma unroll
                for (int j = 0; j < V; ++j) acc[j] += cv[u] * pr[u][j];
            }
        }
    }
    if constexpr (LOSS) {
        lacc = wave_sum_d(lacc);
        if (lane == 0) a.partial[shard] = lacc;
        return;
    }
    if constexpr (GONLY) {
        if (ract) store_row<V, STRIDED>(out + (int64_t)f * R, R, sub, acc);
        return;
    }
    if constexpr (RLOSS) {
        lacc = wave_sum_d(lacc);                 // every lane takes part
        if (lane == 0) a.partial[shard] = lacc;
    }
    const bool single = in_head;                 // whole run is one row
    const int tail_row = cur_row;
    if (single) {
#pragma unroll
        for (int j = 0; j < V; ++j) head[j] = acc[j];
    }
    // join tails to the heads that continue them: segmented scan over slots
    const int prev_tail = __shfl_up(tail_row, LANES);
    const bool link = (slot > 0) && (prev_tail == head_row);
    const bool hflag = !(single && link);
    const uint64_t hm = __ballot(hflag && sub == 0);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int sstart = (63 - __clzll(hm & upto)) / LANES;
    float c[V];
#pragma unroll
    for (int j = 0; j < V; ++j) c[j] = acc[j];
#pragma unroll
    for (int d = 1; d < SW; d <<= 1) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const float t = __shfl_up(c[j], d * LANES);
            if (slot - d >= sstart) c[j] += t;
        }
    }
    float cin[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const float t = __shfl_up(c[j], LANES);
        cin[j] = link ? t : 0.0f;
    }
    const bool next_link = __shfl_down((int)link, LANES) != 0;
    if (ract) {
        if (!single) {
            float h[V];
#pragma unroll
            for (int j = 0; j < V; ++j) h[j] = head[j] + cin[j];
            FLUSH_MID(head_row, h);
        }
        if (slot < SW - 1 && !next_link) FLUSH_MID(tail_row, c);
        if (slot == SW - 1) {
            // the shard's last row: complete, or a boundary partial
            const bool split_after = a.row_ptr[l + 1] > end;
            float *dst;
            if (l == f && split_before) dst = cbase;
            else if (split_after) dst = cbase + (l == f ? 0 : R);
            else dst = out + (int64_t)l * R;
            store_row<V, STRIDED>(dst, R, sub, c);
        }
    }
#undef FLUSH_MID
}

// ---- standalone remap: L_{n+1}[P_n[i]] = L_n[i] -------------------------
// Each block stages one chunk of RB = 256 * RT consecutive records in LDS (RT = 16
// or 24, fewer for wide records so the stage stays within 96 KB), groups them by
// destination 128-byte line (counting sort on the line number modulo 1024),
// then stores them in that order, so that records bound for the same line
// leave in the same store instruction and the L2 combines them into one
// write.  The result does not depend on the store order (every record has
// its own destination).
//

// An L_n record in L_{n+1}'s format (as repack) for records of at most
// three coordinate words, as one bit-string operation (parameters in
// RemapMap) on a 64-bit (W <= 2) or 128-bit (W = 3) integer.
template <int W>
struct RecBits {
    using T = uint64_t;
};
template <>
struct RecBits<3> {
    using T = unsigned __int128;
};

template <int W>
__device__ __forceinline__ Rec<W> repack_bits(const Rec<W> &r, int row, const RemapMap &rm)
{
    static_assert(W <= 3, "three coordinate words at most");
    using T = typename RecBits<W>::T;
    T x = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) x |= (T)r.w[k] << (32 * k);
    constexpr uint32_t B = 8 * sizeof(T);
    const T lowm = rm.ba >= B ? ~(T)0 : ((T)1 << rm.ba) - (T)1;
    const T hm = rm.hi ? ~(T)0 : (T)0;
    const T y = (x & lowm) | (((x >> rm.bh) << rm.bu) & hm) | ((T)(uint32_t)row << rm.bp);
    Rec<W> o;
#pragma unroll
    for (int k = 0; k < W; ++k) o.w[k] = (uint32_t)(y >> (32 * k));
    o.w[W] = r.w[W];
    return o;
}

// Each record also changes format on the way: c_n (recovered from L_n's
// row-start table and the plan's row ids) is stored and c_{n+1} (implied by
// the record's slot in L_{n+1}) dropped.  Wave w of the block reads the
// RT * 64 consecutive positions from base + w * RT * 64 (a "region"), one
// 64-position table block per record step, so that one load per lane brings
// the wave's table entries (read back with readlane), and, when the region
// covers at most 64 rows (nearly always), one more brings all their row ids
// (read back with a lane shuffle), with no load depending on another: with
// one block per CU (its LDS stage), nothing else hides such a chain.  Reads
// stay coalesced (64 consecutive records per load), and the result does not
// depend on which thread moves which record.
// RT records per thread (remap_rt_of in launch.hpp; the host sizes the grid
// and the per-region row ids with the same function).
template <int N, int W, int RT>
__global__ __launch_bounds__(256) void remap_kernel(const uint32_t *__restrict__ rin,
                                                    uint32_t *__restrict__ rout,
                                                    const int32_t *__restrict__ perm,
                                                    int64_t nnz, RemapMap rm)
{
    constexpr int RB = 256 * RT;
    constexpr int NB = 1024;              // buckets
    static_assert(RT + 1 <= 64, "a wave's table entries take one load per lane");
    __shared__ Rec<W> srec[RB];
    __shared__ int32_t sdst[RB];
    __shared__ int32_t cnt[NB];
    const int t = threadIdx.x;
    const int lane = t & 63;
    // XCD-aware chunk order: workgroups are handed to the 8 XCDs round-robin,
    // so block b takes chunk (b % 8) * per + b / 8 and every XCD walks one
    // contiguous range of the tensor.  Records that share a destination line
    // come from neighbouring chunks (consecutive output rows of this mode),
    // so their partial-line writes meet, and combine, in the same L2.
    const int64_t nchunks = (nnz + RB - 1) / RB;
    const int64_t per = (nchunks + 7) / 8;
    const int64_t chunk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (chunk < nchunks) {
        const int64_t base = chunk * RB;
        const int64_t wbase = base + (int64_t)(t >> 6) * RT * 64;   // multiple of 64
        for (int k = t; k < NB; k += 256) cnt[k] = 0;
        // the wave's row ids (plan table) and row-start table entries, one
        // load per lane each, issued before the records: neither depends on
        // another load
        const int rid = rm.rids[(wbase / (RT * 64)) * 64 + lane];
        RowStart ent{0u, 0u, 0u};
        if (lane <= RT) {
            const int64_t b = wbase / 64 + lane;
            ent = row_start_at(rm.rbits, (int)(b < rm.nblk ? b : rm.nblk));
        }
        __syncthreads();
        Rec<W> r[RT];
        int32_t d[RT], pos[RT];
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int64_t i = wbase + k * 64 + lane;
            const bool ok = i < nnz;
            // Read-once streams are loaded non-temporal, so they do not
            // evict the partly written destination lines that wait in L2 for
            // their other records, nor the new layout in the Infinity Cache,
            // which the next MTTKRP reads (12-byte records: that kernel
            // 0.237 -> 0.215 ms).  Records only when they are 8, 12, 16 or
            // 32 bytes: for 20- and 24-byte records non-temporal loads measured
            // 15-45% slower, also when the chunk was first staged so that
            // every line is read once.
            if constexpr ((W + 1) % 4 == 0 || W + 1 <= 3) r[k] = load_rec_nt<W>(rin, ok ? i : 0);
            else r[k] = load_rec<W>(rin, ok ? i : 0);
            d[k] = ok ? __builtin_nontemporal_load(perm + i) : -1;
        }
        // The entries cover the wave's RT blocks and the block after them
        // (past the end: the last entry, which has no bits and the row
        // count).  The wave's row ordinals start at o_first, the row holding
        // its first position; rid holds the ids of rows o_first + lane
        // unless the region covers more than 64 rows (then they are read
        // from the list of nonempty rows).
        const int o_first = __builtin_amdgcn_readlane((int)ent.cnt, 0) +
                            (__builtin_amdgcn_readlane((int)ent.lo, 0) & 1) - 1;
        const bool staged = __builtin_amdgcn_readlane(rid, 0) >= 0;   // wave-uniform
        int row[RT];
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const RowStart e{(uint32_t)__builtin_amdgcn_readlane((int)ent.lo, k),
                             (uint32_t)__builtin_amdgcn_readlane((int)ent.hi, k),
                             (uint32_t)__builtin_amdgcn_readlane((int)ent.cnt, k)};
            bool st;
            const int o = row_ordinal(e, lane, st);   // position wbase + 64k + lane
            if (staged) row[k] = __shfl(rid, o - o_first);
            else row[k] = rm.nrows[(d[k] >= 0) ? o : 0];   // in-range index either way
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            if constexpr (W <= 3) r[k] = repack_bits<W>(r[k], row[k], rm);
            else r[k] = repack<N, W>(r[k], row[k], rm.n, rm.nx, rm.ioff, rm.ooff, rm.msk);
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int b = (d[k] >= 0) ? (int)(((int64_t)d[k] * (W + 1) / 32) & (NB - 1)) : NB - 1;
            pos[k] = atomicAdd(&cnt[b], 1);   // LDS atomic: slot within bucket
            d[k] = (d[k] >= 0) ? d[k] : -1;
            pos[k] |= b << 16;
        }
        __syncthreads();
        // exclusive scan of the bucket counts (4 per thread, then across)
        {
            static_assert(NB == 1024, "scan assumes 4 buckets per thread");
            int c0 = cnt[4 * t], c1 = cnt[4 * t + 1], c2 = cnt[4 * t + 2], c3 = cnt[4 * t + 3];
            int s = c0 + c1 + c2 + c3, x = s;
            const int lane = t & 63, w = t >> 6;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const int y = __shfl_up(x, dd);
                if (lane >= dd) x += y;
            }
            __shared__ int wsum[4];
            if (lane == 63) wsum[w] = x;
            __syncthreads();
            int off = 0;
            for (int k = 0; k < w; ++k) off += wsum[k];
            int e = off + x - s;
            cnt[4 * t] = e; e += c0;
            cnt[4 * t + 1] = e; e += c1;
            cnt[4 * t + 2] = e; e += c2;
            cnt[4 * t + 3] = e;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int slot = cnt[pos[k] >> 16] + (pos[k] & 0xffff);
            srec[slot] = r[k];
            sdst[slot] = d[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int slot = k * 256 + t;
            const int32_t dst = sdst[slot];
            if (dst >= 0) store_rec<W>(rout, dst, srec[slot]);
        }
        __syncthreads();
    }
}

}  // namespace mk
