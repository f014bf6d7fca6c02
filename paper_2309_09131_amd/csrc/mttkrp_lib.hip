// Host side of the C ABI declared in include/mttkrp.h: argument checks,
// workspace carve-up, plan construction (device sorts + host partition
// tables), and the launch sequences of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "als_kernels.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "mttkrp.h"
#include "plan_kernels.hpp"

namespace {

constexpr int DEFAULT_G = 1024;
constexpr int DEFAULT_WORKERS = 256;
constexpr int GRAM_TARGET_BLOCKS = 1024;
constexpr int SEG_VALS = 8192;        // floats a segmented-reduction block stages

// entries per segmented-reduction block
int seg_block(int R) { return std::min(256, SEG_VALS / R); }

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// The integer a C caller passed for an enum parameter, read without an
// enum-typed load (C allows any int there; C++ makes loading a value outside
// the enumeration undefined), so it can be validated first.
template <typename E>
int raw_enum(const E &e)
{
    static_assert(sizeof(E) == sizeof(int), "C enums are int-sized here");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

struct Layout {
    int N;
    int64_t dims[MTTKRP_MAX_MODES];
    int64_t nnz;
    int R;
    int g;
    int workers;
    uint32_t flags;
    int cw;                            // coordinate words per record
    // bit offset of coordinate k in a record of layout L_m (L_m's records
    // omit c_m, implied by the position; loff[m][m] is unused)
    uint32_t loff[MTTKRP_MAX_MODES][MTTKRP_MAX_MODES];
    uint32_t cmask[MTTKRP_MAX_MODES];  // mask of coordinate k, 2^b_k - 1
    uint32_t fw[MTTKRP_MAX_MODES];     // field width of coordinate k (b_k, or 32 unpacked)
    int64_t nblk;                      // row-start table entries - 1 (ceil(nnz / 64))
    bool rsmall[MTTKRP_MAX_MODES];     // remap L_n -> L_{n+1} in its small form
    int64_t nreg[MTTKRP_MAX_MODES];    // its regions (64 * RT positions each)
    int64_t m[MTTKRP_MAX_MODES], k[MTTKRP_MAX_MODES], maxS[MTTKRP_MAX_MODES];
    size_t off_rec[2], off_perm[MTTKRP_MAX_MODES], off_rp[MTTKRP_MAX_MODES];
    size_t off_res[MTTKRP_MAX_MODES];   // resident copy of L_n (MTTKRP_RESIDENT_LAYOUT)
    uint32_t resident;                  // bit n: L_n kept resident
    size_t off_sh[MTTKRP_MAX_MODES], off_ord[MTTKRP_MAX_MODES], off_split[MTTKRP_MAX_MODES];
    size_t off_lpt[MTTKRP_MAX_MODES];
    size_t off_rb[MTTKRP_MAX_MODES];   // row-start table of L_n
    size_t off_nr[MTTKRP_MAX_MODES];   // nonempty rows of mode n
    size_t off_fl[MTTKRP_MAX_MODES];   // first and last row of each shard
    size_t off_rid[MTTKRP_MAX_MODES];  // row ids of each remap region of L_n
    size_t off_xx, off_misc;           // persistent scalars
    size_t off_scratch, scratch_bytes, total;
    // runtime scratch (inside scratch)
    size_t rt_carry[2], rt_partial, rt_G, rt_L, rt_Linv, rt_W, rt_gpart, rt_colsq, rt_lambda_tmp;
    size_t rt_seg[2], rt_segk[2];
    // plan scratch (inside scratch)
    size_t ps_k0, ps_k1, ps_v0, ps_v1, ps_o0, ps_o1, ps_hist, ps_hscan, ps_sums, ps_err;
};

int64_t default_m(int64_t I, int workers)
{
    if (I < workers) return 1;
    int64_t q = 1;
    int64_t m = (I + workers - 1) / workers;
    if (m > 16000) {
        q = (I + (int64_t)workers * 16000 - 1) / ((int64_t)workers * 16000);
        m = (I + q * workers - 1) / (q * workers);
    }
    return m;
}

mttkrp_status compute_layout(int N, const int64_t *dims, int64_t nnz, int R,
                             const mttkrp_plan_opts *opts, Layout *L, std::string *why)
{
    if (N < 2 || N > MTTKRP_MAX_MODES) { *why = "nmodes must be in [2, 8]"; return MTTKRP_EINVAL; }
    if (!dims) { *why = "dims is NULL"; return MTTKRP_EINVAL; }
    if (R < 1 || R > MTTKRP_MAX_RANK) { *why = "rank must be in [1, 256]"; return MTTKRP_EINVAL; }
    // the kernels index nonzeros with 32-bit integers and may form indices
    // up to a few hundred past the end of a shard before clamping them
    if (nnz < 0 || nnz > MTTKRP_MAX_NNZ) {
        *why = "nnz must be in [0, " + std::to_string((long long)MTTKRP_MAX_NNZ) + "]";
        return MTTKRP_EINVAL;
    }
    memset(L, 0, sizeof(*L));
    L->N = N; L->nnz = nnz; L->R = R;
    L->g = (opts && opts->g > 0) ? opts->g : DEFAULT_G;
    L->workers = (opts && opts->workers > 0) ? opts->workers : DEFAULT_WORKERS;
    L->flags = opts ? opts->flags : 0u;
    if (opts && opts->g < 0) { *why = "g must be >= 0"; return MTTKRP_EINVAL; }
    L->resident = (L->flags >> 16) & 0xffu;
    if (L->resident >> N) {
        *why = "MTTKRP_RESIDENT_LAYOUT names a mode >= nmodes";
        return MTTKRP_EINVAL;
    }
    for (int n = 0; n < N; ++n) {
        if (dims[n] < 1 || dims[n] >= (int64_t(1) << 31)) {
            *why = "every dimension must be in [1, 2^31)";
            return MTTKRP_EINVAL;
        }
        L->dims[n] = dims[n];
        if (opts && opts->m[n] < 0) { *why = "m[n] must be >= 0"; return MTTKRP_EINVAL; }
        L->m[n] = (opts && opts->m[n] > 0) ? opts->m[n] : default_m(dims[n], L->workers);
        if (L->m[n] > dims[n]) L->m[n] = dims[n];
        L->k[n] = (dims[n] + L->m[n] - 1) / L->m[n];
        L->maxS[n] = (nnz + L->g - 1) / L->g + L->k[n];
    }
    // Record format of layout L_m: the coordinates other than c_m (which the
    // position in L_m implies, through the row-start table) bit-packed in
    // mode order, b_k = bit length of I_k - 1 bits each (a coordinate may
    // straddle two words); or one word per coordinate when the plan asks for
    // it.  A 0-bit coordinate (I_k = 1) sits at offset 0 with an empty mask.
    // Every layout uses the same cw: the widest layout's words, rounded up
    // to the narrowest compiled width.
    const bool unpacked = (L->flags & MTTKRP_UNPACKED_RECORDS) != 0;
    int bits[MTTKRP_MAX_MODES];
    for (int n = 0; n < N; ++n) {
        int b = 0;
        while ((int64_t(1) << b) < dims[n]) ++b;
        bits[n] = b;
        L->cmask[n] = b ? (uint32_t)((uint64_t(1) << b) - 1) : 0u;
        L->fw[n] = unpacked ? 32u : (uint32_t)b;
    }
    int words = 1;
    for (int m = 0; m < N; ++m) {
        int tot = 0, slot = 0;
        for (int k = 0; k < N; ++k) {
            if (k == m) { L->loff[m][k] = 0u; continue; }
            L->loff[m][k] = unpacked ? 32u * slot : (bits[k] ? (uint32_t)tot : 0u);
            tot += bits[k];
            ++slot;
        }
        words = std::max(words, (tot + 31) / 32);
    }
    L->cw = unpacked ? N - 1 : std::max(mk::rec_wmin(N), words);
    L->nblk = (nnz + 63) / 64;
    // one region per wave of each remap block (4 waves of RT * 64 records)
    for (int n = 0; n < N; ++n) {
        L->rsmall[n] = dims[(n + 1) % N] <= mk::REMAP_SMALL_ROWS;
        const int64_t rb = 256 * (int64_t)mk::remap_rt_of(L->cw, L->rsmall[n]);
        L->nreg[n] = 4 * ((nnz + rb - 1) / rb);
    }
    const int NW = L->cw + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L->off_rec[0] = take((size_t)nnz * NW * 4);
    L->off_rec[1] = take((size_t)nnz * NW * 4);
    for (int n = 0; n < N; ++n)
        L->off_res[n] = (L->resident >> n & 1u) ? take((size_t)nnz * NW * 4) : 0;
    for (int n = 0; n < N; ++n) L->off_perm[n] = take((size_t)nnz * 4);
    for (int n = 0; n < N; ++n) L->off_rp[n] = take((size_t)(dims[n] + 1) * 4);
    int64_t maxS = 0;
    for (int n = 0; n < N; ++n) {
        L->off_sh[n] = take((size_t)L->maxS[n] * 12);
        L->off_ord[n] = take((size_t)L->maxS[n] * 4);
        L->off_split[n] = take((size_t)L->maxS[n] * 16);
        L->off_lpt[n] = take((size_t)L->k[n] * 4);
        L->off_rb[n] = take((size_t)(L->nblk + 1) * mk::RS_WORDS * 4);
        L->off_nr[n] = take((size_t)(std::min<int64_t>(dims[n], std::max<int64_t>(nnz, 1)) + 1) * 4);
        L->off_fl[n] = take((size_t)L->maxS[n] * 8);
        L->off_rid[n] = take((size_t)std::max<int64_t>(L->nreg[n], 1) * 64 * 4);
        maxS = std::max(maxS, L->maxS[n]);
    }
    L->off_xx = take(64);
    L->off_misc = take(64);                    // ridge counter, fail flag
    L->off_scratch = off;
    // runtime scratch
    size_t r0 = 0;
    auto rtake = [&](size_t bytes) { size_t o = r0; r0 = align_up(r0 + bytes); return o; };
    L->rt_carry[0] = rtake((size_t)maxS * 2 * R * 4);   // two: modes alternate
    L->rt_carry[1] = rtake((size_t)maxS * 2 * R * 4);
    L->rt_partial = rtake((size_t)std::max<int64_t>(maxS, 4096) * 8);
    L->rt_G = rtake((size_t)N * R * R * 8);
    L->rt_L = rtake((size_t)R * R * 8);
    L->rt_Linv = rtake((size_t)R * R * 8);
    L->rt_W = rtake((size_t)R * R * 8);
    L->rt_gpart = rtake((size_t)GRAM_TARGET_BLOCKS * 256 * 8 + (size_t)R * R * 8);
    L->rt_colsq = rtake((size_t)als::APPLY_BLOCKS * R * 8);
    L->rt_lambda_tmp = rtake((size_t)R * 8 + 64);
    // level 0 has at most 2*maxS entries; each level emits 2 per block
    const int64_t seg_entries = 2 * ((2 * maxS + seg_block(R) - 1) / seg_block(R)) + 8;
    L->rt_seg[0] = rtake((size_t)seg_entries * R * 4);
    L->rt_seg[1] = rtake((size_t)seg_entries * R * 4);
    L->rt_segk[0] = rtake((size_t)seg_entries * 4);
    L->rt_segk[1] = rtake((size_t)seg_entries * 4);
    // plan scratch
    size_t p0 = 0;
    auto ptake = [&](size_t bytes) { size_t o = p0; p0 = align_up(p0 + bytes); return o; };
    const int64_t ntiles = (nnz + plan::TILE - 1) / plan::TILE;
    const int64_t hlen = 256 * std::max<int64_t>(ntiles, 1);
    L->ps_k0 = ptake((size_t)nnz * 4);
    L->ps_k1 = ptake((size_t)nnz * 4);
    L->ps_v0 = ptake((size_t)nnz * 4);
    L->ps_v1 = ptake((size_t)nnz * 4);
    L->ps_o0 = ptake((size_t)nnz * 4);
    L->ps_o1 = ptake((size_t)nnz * 4);
    L->ps_hist = ptake((size_t)hlen * 4);
    L->ps_hscan = ptake((size_t)hlen * 4);
    L->ps_sums = ptake((size_t)((hlen + plan::SCAN_CHUNK - 1) / plan::SCAN_CHUNK + 1) * 4);
    L->ps_err = ptake(64);
    L->scratch_bytes = std::max(r0, p0);
    L->total = L->off_scratch + L->scratch_bytes;
    return MTTKRP_OK;
}

struct ProfEvent { hipEvent_t a, b; int mode; int kernel; };

}  // namespace

struct mttkrp_plan_s {
    Layout L;
    char *ws = nullptr;
    int cur = 0;            // layout the tensor is in
    int buf = 0;            // record buffer holding it: 0, 1 (work) or 2 + n (resident L_n)
    int64_t nshards[MTTKRP_MAX_MODES] = {};
    int64_t nsplit[MTTKRP_MAX_MODES] = {};   // rows split across shards
    int64_t npart[MTTKRP_MAX_MODES] = {};    // their boundary partials (P0)
    int64_t nempty[MTTKRP_MAX_MODES] = {};
    std::string err;
    bool prof = false;
    std::vector<ProfEvent> events;
    std::vector<hipEvent_t> pool;
    // second stream for the boundary-partial reduction, overlapped with the
    // remap kernel; carry buffers alternate between consecutive passes
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_seg[2] = {nullptr, nullptr};
    hipEvent_t ev_als = nullptr;   // CP-ALS: mode update forked after its MTTKRP
    bool seg_pending[2] = {false, false};
    // output range each pending reduction writes (callers may pass one
    // buffer for several passes: a later pass must not start before it)
    const char *seg_out[2] = {nullptr, nullptr};
    size_t seg_out_bytes[2] = {0, 0};
    bool aux_pending = false;
    int carry_sel = 0;

    uint32_t *rec(int b)
    {
        return reinterpret_cast<uint32_t *>(ws + (b < 2 ? L.off_rec[b] : L.off_res[b - 2]));
    }
    // the buffer that holds L_to after the tensor moves there from buffer
    // `from`: its resident copy, else the work buffer that `from` is not
    int next_buf(int from, int to) const
    {
        if (L.resident >> to & 1u) return 2 + to;
        return from == 0 ? 1 : 0;
    }
    int32_t *perm(int n) { return reinterpret_cast<int32_t *>(ws + L.off_perm[n]); }
    int32_t *rp(int n) { return reinterpret_cast<int32_t *>(ws + L.off_rp[n]); }
    int32_t *sh(int n) { return reinterpret_cast<int32_t *>(ws + L.off_sh[n]); }
    int32_t *ord(int n) { return reinterpret_cast<int32_t *>(ws + L.off_ord[n]); }
    int32_t *split(int n) { return reinterpret_cast<int32_t *>(ws + L.off_split[n]); }
    int32_t *lpt(int n) { return reinterpret_cast<int32_t *>(ws + L.off_lpt[n]); }
    uint32_t *rb(int n) { return reinterpret_cast<uint32_t *>(ws + L.off_rb[n]); }
    int32_t *nr(int n) { return reinterpret_cast<int32_t *>(ws + L.off_nr[n]); }
    int32_t *fl(int n) { return reinterpret_cast<int32_t *>(ws + L.off_fl[n]); }
    int32_t *rid(int n) { return reinterpret_cast<int32_t *>(ws + L.off_rid[n]); }
    // the standalone remap's map from L_n to L_{n+1}
    mk::RemapMap remap_map(int n)
    {
        mk::RemapMap m;
        memset(&m, 0, sizeof(m));
        const int nx = (n + 1) % L.N;
        for (int k = 0; k < L.N; ++k) {
            m.ioff[k] = L.loff[n][k];
            m.ooff[k] = L.loff[nx][k];
            m.msk[k] = L.cmask[k];
        }
        m.rbits = rb(n);
        m.nrows = nr(n);
        m.rids = rid(n);
        m.nblk = (int32_t)L.nblk;
        m.n = n;
        m.nx = nx;
        m.small = L.rsmall[n] ? 1 : 0;
        // The move as a bit string (records of at most two words).  L_n
        // stores the modes other than n in mode order, L_{n+1} those other
        // than n + 1: the fields below bit a stay, c_{n+1}'s (win bits at a)
        // is dropped, the fields above move to a + gap, c_n goes to bit rpos.
        uint32_t a = 0, win, gap, rpos;
        if (nx == 0) {        // c_0 leaves the bottom, c_{N-1} joins the top
            win = L.fw[0];
            gap = 0;
            rpos = 0;
            for (int k = 1; k < L.N - 1; ++k) rpos += L.fw[k];
        } else {              // c_{n+1}'s field becomes c_n's
            for (int k = 0; k < n; ++k) a += L.fw[k];
            win = L.fw[nx];
            gap = L.fw[n];
            rpos = a;
        }
        // the kernels use this form for W <= 3, on a B-bit integer
        const uint32_t B = L.cw <= 2 ? 64u : 128u;
        const uint32_t top = 32u * (uint32_t)L.cw;      // stored coordinate bits
        m.ba = a;                                       // a >= B: every bit below
        m.hi = (a + win < top && a + gap < B) ? 1u : 0u;
        m.bh = m.hi ? a + win : 0u;
        m.bu = m.hi ? a + gap : 0u;
        m.bp = std::min(rpos, B - 1);   // beyond B - 1 only for a 0-bit c_n (c_n = 0)
        return m;
    }
    double *xx() { return reinterpret_cast<double *>(ws + L.off_xx); }
    int32_t *ridge() { return reinterpret_cast<int32_t *>(ws + L.off_misc); }
    int32_t *fail() { return reinterpret_cast<int32_t *>(ws + L.off_misc) + 1; }
    double *fit_slot() { return reinterpret_cast<double *>(ws + L.off_misc) + 1; }
    template <typename T> T *rt(size_t o) { return reinterpret_cast<T *>(ws + L.off_scratch + o); }
};

static std::string g_last_error;

#define HIPCHK(p, call)                                                        \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            set_err((p), std::string(#call) + ": " + hipGetErrorString(e_));   \
            return MTTKRP_EHIP;                                                \
        }                                                                      \
    } while (0)

static void set_err(mttkrp_plan_t p, const std::string &s)
{
    if (p) p->err = s;
    else g_last_error = s;
}

static mttkrp_status fail(mttkrp_plan_t p, mttkrp_status st, const std::string &s)
{
    set_err(p, s);
    return st;
}

static unsigned grid_for(int64_t n, int per = 256, unsigned cap = 65536)
{
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

// ---------------------------------------------------------------- kernels
// launch dispatch by mode count

static hipError_t launch_mttkrp_any(int N, const mk::Args &a, int bf16, mk::LaneCfg c, int kind,
                                    unsigned grid, hipStream_t s)
{
    switch (N) {
    case 2: return mk::launch_mttkrp<2>(a, bf16, c, kind, grid, s);
    case 3: return mk::launch_mttkrp<3>(a, bf16, c, kind, grid, s);
    case 4: return mk::launch_mttkrp<4>(a, bf16, c, kind, grid, s);
    case 5: return mk::launch_mttkrp<5>(a, bf16, c, kind, grid, s);
    case 6: return mk::launch_mttkrp<6>(a, bf16, c, kind, grid, s);
    case 7: return mk::launch_mttkrp<7>(a, bf16, c, kind, grid, s);
    case 8: return mk::launch_mttkrp<8>(a, bf16, c, kind, grid, s);
    }
    return hipErrorInvalidValue;
}

// L_n (in rin) -> L_{n+1} (in rout)
static hipError_t launch_remap_any(mttkrp_plan_t p, int n, const uint32_t *rin, uint32_t *rout,
                                   hipStream_t s)
{
    const Layout &L = p->L;
    const mk::RemapMap rm = p->remap_map(n);
    const int32_t *perm = p->perm(n);
    const int64_t nnz = L.nnz;
    const int cw = L.cw;
    switch (L.N) {
    case 2: return mk::launch_remap<2>(rin, rout, perm, nnz, cw, rm, s);
    case 3: return mk::launch_remap<3>(rin, rout, perm, nnz, cw, rm, s);
    case 4: return mk::launch_remap<4>(rin, rout, perm, nnz, cw, rm, s);
    case 5: return mk::launch_remap<5>(rin, rout, perm, nnz, cw, rm, s);
    case 6: return mk::launch_remap<6>(rin, rout, perm, nnz, cw, rm, s);
    case 7: return mk::launch_remap<7>(rin, rout, perm, nnz, cw, rm, s);
    case 8: return mk::launch_remap<8>(rin, rout, perm, nnz, cw, rm, s);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_pack_any(const Layout &L, const int32_t *idx, const float *vals,
                                  const int32_t *o, uint32_t *rec, hipStream_t s)
{
    mk::PackMap pm;
    for (int n = 0; n < 8; ++n) pm.off[n] = n < L.N ? L.loff[0][n] : 0u;
    pm.skip = 0;
    const int64_t nnz = L.nnz;
    switch (L.N) {
    case 2: return mk::launch_pack<2>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 3: return mk::launch_pack<3>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 4: return mk::launch_pack<4>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 5: return mk::launch_pack<5>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 6: return mk::launch_pack<6>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 7: return mk::launch_pack<7>(idx, vals, o, nnz, rec, L.cw, pm, s);
    case 8: return mk::launch_pack<8>(idx, vals, o, nnz, rec, L.cw, pm, s);
    }
    return hipErrorInvalidValue;
}

// Zero fill and carry fix-up (mode-count independent).
__global__ void fill_zero_kernel(float *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Deterministic segmented reduction of the shard boundary partials of rows
// split across shards (one level).  Entries are R-float vectors with sorted
// row keys (level 0: read through `ids` from the per-shard partial slots).
// Block b takes entries [b*B, (b+1)*B), B = seg_block(R): they are first
// staged in LDS with coalesced loads; then slots of RL lanes walk runs in
// order; rows wholly inside the block are written to `out`; the block's
// first and last rows go to the next level as two entries (or to `out` when
// this is the last level).  Fixed partition and order: bit-exact reruns.

__global__ __launch_bounds__(256) void seg_reduce_kernel(const float *__restrict__ src,
                                                         const int32_t *__restrict__ ids,
                                                         const int32_t *__restrict__ keys,
                                                         int64_t P, int B, int R, int RL,
                                                         float *__restrict__ out,
                                                         float *__restrict__ next,
                                                         int32_t *__restrict__ next_keys,
                                                         int last_level)
{
    __shared__ int32_t s_head[256], s_tail[256], s_single[256];
    __shared__ float s_hsum[2 * 256];          // [SL][R] heads, then tails (SL*R <= 256)
    __shared__ float s_val[SEG_VALS];
    __shared__ int32_t s_key[256];
    const int SL = 256 / RL;
    const int r = threadIdx.x % RL, slot = threadIdx.x / RL;
    const int64_t b0 = (int64_t)blockIdx.x * B;
    const int64_t b1 = (b0 + B < P) ? b0 + B : P;
    const int cnt = (int)(b1 - b0);
    if ((int)threadIdx.x < cnt) s_key[threadIdx.x] = keys[b0 + threadIdx.x];
    // eight loads in flight per thread (clamped indices, no branch around
    // the loads), then the LDS writes
    const int nv = cnt * R;
    for (int x0 = 0; x0 < nv; x0 += 256 * 8) {
        float v[8];
        int64_t ent[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int x = x0 + j * 256 + (int)threadIdx.x;
            x = x < nv ? x : nv - 1;
            const int e = x / R;
            ent[j] = ids ? (int64_t)ids[b0 + e] : b0 + e;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int x = x0 + j * 256 + (int)threadIdx.x;
            x = x < nv ? x : nv - 1;
            v[j] = src[ent[j] * R + (x - (x / R) * R)];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int x = x0 + j * 256 + (int)threadIdx.x;
            if (x < nv) s_val[x] = v[j];
        }
    }
    __syncthreads();
    const int run = (B + SL - 1) / SL;
    const int s0 = slot * run;
    const int s1 = (s0 + run < cnt) ? s0 + run : cnt;
    const int first_row = s_key[0];
    float *hs = s_hsum;
    float *ts = s_hsum + SL * R;
    // per-slot sequential pass
    int cur = -1, head = -1;
    bool single = true;
    float acc = 0.0f, hsum = 0.0f;
    for (int e = s0; e < s1; ++e) {
        const int row = s_key[e];
        const float v = (r < R) ? s_val[e * R + r] : 0.0f;
        if (cur < 0) {
            cur = head = row;
        } else if (row != cur) {
            if (single) {
                hsum = acc;
                single = false;
            } else if (r < R) {
                out[(int64_t)cur * R + r] = acc;      // interior row
            }
            acc = 0.0f;
            cur = row;
        }
        acc += v;
    }
    if (single) hsum = acc;
    if (r == 0) {
        s_head[slot] = head;
        s_tail[slot] = cur;
        s_single[slot] = single ? 1 : 0;
    }
    if (r < R) {
        hs[slot * R + r] = hsum;
        ts[slot * R + r] = acc;
    }
    __syncthreads();
    // one group of RL lanes joins the slots in order
    if (slot != 0) return;
    int row = -1;
    float sum = 0.0f;
    auto flush = [&](int rw, float v) {
        if (rw == first_row && !last_level) {
            if (r < R) next[(2 * (int64_t)blockIdx.x) * R + r] = v;
        } else if (r < R) {
            out[(int64_t)rw * R + r] = v;
        }
    };
    bool first_flushed = false;
    for (int k = 0; k < SL; ++k) {
        const int h = s_head[k];
        if (h < 0) continue;                      // empty slot
        const float hv = (r < R) ? hs[k * R + r] : 0.0f;
        if (row == h) {
            sum += hv;
        } else {
            if (row >= 0) {
                flush(row, sum);
                first_flushed |= (row == first_row);
            }
            row = h;
            sum = hv;
        }
        if (!s_single[k]) {
            flush(row, sum);
            first_flushed |= (row == first_row);
            row = s_tail[k];
            sum = (r < R) ? ts[k * R + r] : 0.0f;
        }
    }
    // the block's last row (may equal its first row)
    if (last_level) {
        if (r < R) out[(int64_t)row * R + r] = sum;
    } else {
        float *e0 = next + (2 * (int64_t)blockIdx.x) * R;
        float *e1 = e0 + R;
        if (row == first_row && !first_flushed) {
            if (r < R) { e0[r] = sum; e1[r] = 0.0f; }
        } else if (r < R) {
            e1[r] = sum;
        }
        if (r == 0) {
            next_keys[2 * blockIdx.x] = first_row;
            next_keys[2 * blockIdx.x + 1] = row;
        }
    }
}

// ---------------------------------------------------------------- helpers

static int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static mk::LaneCfg lane_cfg(int R, mttkrp_dtype fdt, const void *const *facs, int N,
                            const float *out)
{
    // FP32 rows with two or three modes: lanes per nonzero = R / 8, each
    // reading 32 bytes (two 16-byte loads).  From four modes on, and for
    // BF16 rows: 16 bytes per lane (R / 4 or R / 8 lanes), which needs fewer
    // registers per nonzero (4-mode FP32 kernel: 127 against 187 VGPRs, 4
    // waves per SIMD instead of 2).  Measured, FP32 sweeps with 16-byte
    // against 32-byte lanes: 4 modes R 32 10.18 against 10.42 ms, 5 modes R
    // 16 23.96 against 25.33 ms, 3 modes R 32 1.05 against 0.99 ms and R 64
    // 1.61 against 1.46 ms (the 3-mode R 64 loss step within 1%).  Otherwise
    // the strided form, for ranks that are not a multiple of the vector
    // width.
    const bool bf = fdt == MTTKRP_BF16;
    const int V16 = bf ? 8 : 4;                  // elements per 16 bytes
    bool ok = (R % V16 == 0) && (out == nullptr || aligned16(out));
    for (int w = 0; w < N && ok; ++w)
        if (facs[w] && !aligned16(facs[w])) ok = false;
    if (ok && !bf && N <= 3 && R % 8 == 0 && next_pow2(R / 8) <= 32)
        return mk::LaneCfg{next_pow2(R / 8), 2, false};
    if (ok && next_pow2(R / V16) <= 64) return mk::LaneCfg{next_pow2(R / V16), 1, false};
    return mk::LaneCfg{64, (R + 63) / 64, true};
}

// Stable LSD radix sort of (keys, vals) pairs by the low `bits` of the key.
// Input in (k0, v0); returns which buffer pair holds the result (0 or 1).
static mttkrp_status radix_sort(mttkrp_plan_t p, int32_t *k0, int32_t *v0, int32_t *k1,
                                int32_t *v1, int64_t n, int bits, hipStream_t s, int *which)
{
    const Layout &L = p->L;
    const int64_t ntiles = (n + plan::TILE - 1) / plan::TILE;
    const int64_t hlen = 256 * ntiles;
    int32_t *hist = p->rt<int32_t>(L.ps_hist);
    int32_t *hscan = p->rt<int32_t>(L.ps_hscan);
    int32_t *sums = p->rt<int32_t>(L.ps_sums);
    const int64_t nchunks = (hlen + plan::SCAN_CHUNK - 1) / plan::SCAN_CHUNK;
    int cur = 0;
    int32_t *K[2] = {k0, k1}, *Vv[2] = {v0, v1};
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(plan::radix_upsweep, dim3((unsigned)ntiles), dim3(256), 0, s, K[cur],
                           n, shift, hist, (int)ntiles);
        hipLaunchKernelGGL(plan::scan_reduce, dim3((unsigned)nchunks), dim3(256), 0, s, hist,
                           hlen, sums);
        hipLaunchKernelGGL(plan::scan_sums, dim3(1), dim3(256), 0, s, sums, nchunks);
        hipLaunchKernelGGL(plan::scan_apply, dim3((unsigned)nchunks), dim3(256), 0, s, hist, hlen,
                           sums, hscan);
        hipLaunchKernelGGL(plan::radix_scatter_tile, dim3((unsigned)ntiles), dim3(256), 0, s,
                           K[cur], Vv[cur], n, shift, hscan, (int)ntiles, K[cur ^ 1],
                           Vv[cur ^ 1]);
        HIPCHK(p, hipGetLastError());
        cur ^= 1;
    }
    *which = cur;
    return MTTKRP_OK;
}

static int key_bits(int64_t I)
{
    int b = 0;
    while ((int64_t(1) << b) < I) ++b;
    return b;
}

// Host partition tables of one mode from its row pointers (Sec. III-A, IV-A).
static void build_tables(const Layout &L, int n, const std::vector<int32_t> &rp,
                         std::vector<int32_t> &shards, std::vector<int32_t> &order,
                         std::vector<int32_t> &split, std::vector<int32_t> &lpt_bin,
                         std::vector<int32_t> &fl, int64_t *nempty, int64_t *nsplit_rows)
{
    const int64_t I = L.dims[n], m = L.m[n], k = L.k[n], g = L.g;
    std::vector<int64_t> ss_first(k), ss_cnt(k);
    shards.clear();
    for (int64_t j = 0; j < k; ++j) {
        const int64_t lo = j * m, hi = std::min(I, (j + 1) * m);
        const int64_t a = rp[lo], b = rp[hi];
        ss_first[j] = (int64_t)shards.size() / 3;
        ss_cnt[j] = (b - a + g - 1) / g;
        for (int64_t q = 0; q < ss_cnt[j]; ++q) {
            shards.push_back((int32_t)(a + q * g));
            shards.push_back((int32_t)std::min<int64_t>(g, b - a - q * g));
            shards.push_back((int32_t)j);
        }
    }
    const int64_t S = (int64_t)shards.size() / 3;
    // longest-first scheduling of super-shards over `workers` bins
    std::vector<int64_t> ord(k);
    for (int64_t j = 0; j < k; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int64_t x, int64_t y) { return ss_cnt[x] > ss_cnt[y]; });
    std::vector<int64_t> load(L.workers, 0);
    lpt_bin.assign(k, 0);
    for (int64_t a = 0; a < k; ++a) {
        int best = 0;
        for (int i = 1; i < L.workers; ++i)
            if (load[i] < load[best]) best = i;
        lpt_bin[ord[a]] = best;
        load[best] += ss_cnt[ord[a]];
    }
    order.clear();
    if (L.flags & MTTKRP_NATURAL_ORDER) {
        for (int64_t s = 0; s < S; ++s) order.push_back((int32_t)s);
    } else {
        for (int64_t a = 0; a < k; ++a)
            for (int64_t q = 0; q < ss_cnt[ord[a]]; ++q)
                order.push_back((int32_t)(ss_first[ord[a]] + q));
    }
    // rows split across consecutive shards, flattened for the segmented
    // reduction: for each such row, the partial slots (2*shard + entry) of the
    // shards it spans, in shard order, keyed by the row
    auto row_of = [&](int64_t pos) {   // row r with rp[r] <= pos < rp[r+1]
        auto it = std::upper_bound(rp.begin(), rp.end(), (int32_t)pos);
        return (int64_t)(it - rp.begin()) - 1;
    };
    std::vector<int32_t> ids, keys;
    int64_t rows_split = 0;
    fl.resize(2 * S);
    for (int64_t s = 0; s < S; ++s) {
        const int64_t st = shards[3 * s], en = st + shards[3 * s + 1];
        const int64_t f = row_of(st), l = row_of(en - 1);
        fl[2 * s] = (int32_t)f;
        fl[2 * s + 1] = (int32_t)l;
        const bool sb = rp[f] < st, sa = rp[l + 1] > en;
        if (sb) {                       // continues a split row: entry 0
            ids.push_back((int32_t)(2 * s));
            keys.push_back((int32_t)f);
        }
        if (sa && !(l == f && sb)) {    // opens a split row
            ids.push_back((int32_t)(2 * s + (l == f ? 0 : 1)));
            keys.push_back((int32_t)l);
            ++rows_split;
        }
    }
    split.assign(ids.begin(), ids.end());
    split.insert(split.end(), keys.begin(), keys.end());
    *nsplit_rows = rows_split;
    int64_t ne = 0;
    for (int64_t r = 0; r < I; ++r) ne += (rp[r] == rp[r + 1]);
    *nempty = ne;
}

// Row-start table of L_n and the list of its nonempty rows, from the row
// pointers (table layout in launch.hpp).  Entry nblk (one past the last
// block holding a position) carries the total row count and no bits.
static void build_row_starts(const Layout &L, int n, const std::vector<int32_t> &rp,
                             std::vector<uint32_t> &tab, std::vector<int32_t> &rows,
                             std::vector<int32_t> &rids)
{
    const int64_t I = L.dims[n], nb = L.nblk;
    tab.assign((size_t)(nb + 1) * mk::RS_WORDS, 0u);
    rows.clear();
    for (int64_t r = 0; r < I; ++r) {
        if (rp[r] == rp[r + 1]) continue;
        const int64_t e = rp[r];
        tab[(size_t)(e >> 6) * mk::RS_WORDS + ((e >> 5) & 1)] |= 1u << (e & 31);
        rows.push_back((int32_t)r);
    }
    uint32_t c = 0;
    for (int64_t b = 0; b <= nb; ++b) {
        uint32_t *t = &tab[(size_t)b * mk::RS_WORDS];
        t[2] = c;
        c += (uint32_t)(__builtin_popcount(t[0]) + __builtin_popcount(t[1]));
    }
    const int64_t total = (int64_t)rows.size();
    rows.push_back(rows.empty() ? 0 : rows.back());   // one padding entry
    // row ids of each remap region: rows o_first .. o_first + 63 (the last
    // repeated), or -1 first when more than 64 rows meet the region
    const int64_t reg = 64 * (int64_t)mk::remap_rt_of(L.cw, L.rsmall[n]), nnz = L.nnz;
    rids.assign((size_t)std::max<int64_t>(L.nreg[n], 1) * 64, 0);
    for (int64_t r = 0; r < L.nreg[n]; ++r) {
        const int64_t P = r * reg;
        if (P >= nnz) continue;
        const uint32_t *t = &tab[(size_t)(P >> 6) * mk::RS_WORDS];
        const int64_t o_first = (int64_t)t[2] + (t[0] & 1u) - 1;
        const int64_t pe = std::min(P + reg, nnz);
        const int64_t o_end = pe == nnz ? total : (int64_t)tab[(size_t)(pe >> 6) * mk::RS_WORDS + 2];
        int32_t *d = &rids[(size_t)r * 64];
        if (o_end - o_first > 64) {
            d[0] = -1;
            continue;
        }
        for (int q = 0; q < 64; ++q) d[q] = rows[(size_t)std::min(o_first + q, o_end - 1)];
    }
}

static mttkrp_status check_factors(mttkrp_plan_t p, const void *const *f, int skip_ok, int mode,
                                   const mttkrp_dtype &fdt)
{
    if (!f) return fail(p, MTTKRP_EINVAL, "factor pointer array is NULL");
    const int dt = raw_enum(fdt);               // validated before any enum use
    if (dt != MTTKRP_F32 && dt != MTTKRP_BF16) return fail(p, MTTKRP_EINVAL, "bad dtype");
    for (int w = 0; w < p->L.N; ++w)
        if (!f[w] && !(skip_ok && w == mode))
            return fail(p, MTTKRP_EINVAL, "factor pointer is NULL for mode " + std::to_string(w));
    return MTTKRP_OK;
}

static hipEvent_t take_event(mttkrp_plan_t p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Remap kernel run: L_cur -> L_cur+1.
static hipEvent_t take_event(mttkrp_plan_t p);

static mttkrp_status remap_step(mttkrp_plan_t p, hipStream_t s)
{
    const Layout &L = p->L;
    ProfEvent ev{nullptr, nullptr, p->cur, 1};
    if (p->prof) {
        ev.a = take_event(p);
        ev.b = take_event(p);
    }
    const int nx = (p->cur + 1) % L.N;
    const int dst = p->next_buf(p->buf, nx);
    if (dst >= 2) {
        // L_nx is resident: nothing to move
        if (ev.a) p->pool.push_back(ev.a);
        if (ev.b) p->pool.push_back(ev.b);
        p->buf = dst;
        p->cur = nx;
        return MTTKRP_OK;
    }
    if (ev.a) HIPCHK(p, hipEventRecord(ev.a, s));
    HIPCHK(p, launch_remap_any(p, p->cur, p->rec(p->buf), p->rec(dst), s));
    if (p->prof) {
        if (ev.b) HIPCHK(p, hipEventRecord(ev.b, s));
        p->events.push_back(ev);
    }
    p->buf = dst;
    p->cur = nx;
    return MTTKRP_OK;
}

static mttkrp_status ensure_aux(mttkrp_plan_t p)
{
    if (p->aux) return MTTKRP_OK;
    HIPCHK(p, hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));   // default priority
    HIPCHK(p, hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->ev_seg[0], hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->ev_seg[1], hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->ev_als, hipEventDisableTiming));
    return MTTKRP_OK;
}

// Make `s` wait for everything enqueued on the auxiliary stream so far.
static mttkrp_status join_aux(mttkrp_plan_t p, hipStream_t s)
{
    if (!p->aux_pending) return MTTKRP_OK;
    HIPCHK(p, hipEventRecord(p->ev_join, p->aux));
    HIPCHK(p, hipStreamWaitEvent(s, p->ev_join, 0));
    p->aux_pending = false;
    p->seg_pending[0] = p->seg_pending[1] = false;
    return MTTKRP_OK;
}

// One MTTKRP-family pass over the current layout (mode == p->cur).  The
// reduction of rows split across shards runs on the auxiliary stream beside
// the remap kernel; callers join it before `out` is read on `s`.
static mttkrp_status run_pass(mttkrp_plan_t p, const void *const *facs, mttkrp_dtype fdt,
                              float *out, bool fuse, int kind, const double *gscale,
                              hipStream_t s)
{
    const Layout &L = p->L;
    const int n = p->cur;
    const int64_t rows = L.dims[n];
    if (kind != mk::KIND_LOSS) {
        // a pending reduction of an earlier pass that writes into this
        // pass's output range must finish first
        const char *o0 = reinterpret_cast<const char *>(out);
        const size_t ob = (size_t)rows * L.R * sizeof(float);
        for (int b = 0; b < 2; ++b)
            if (p->seg_pending[b] && o0 < p->seg_out[b] + p->seg_out_bytes[b] &&
                p->seg_out[b] < o0 + ob) {
                HIPCHK(p, hipStreamWaitEvent(s, p->ev_seg[b], 0));
                p->seg_pending[b] = false;
            }
    }
    if (kind != mk::KIND_LOSS && (p->nempty[n] > 0 || L.nnz == 0))
        hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(rows * L.R)), dim3(256), 0, s, out,
                           rows * L.R);
    if (L.nnz == 0) {
        HIPCHK(p, hipGetLastError());
        if (fuse) {
            p->buf = p->next_buf(p->buf, (n + 1) % L.N);
            p->cur = (n + 1) % L.N;
        }
        return MTTKRP_OK;
    }
    mk::Args a;
    memset(&a, 0, sizeof(a));
    // remap inside the MTTKRP kernel only when the plan asks for it; by
    // default the remap runs as its own kernel right after (faster here)
    const bool infuse = fuse && (L.flags & MTTKRP_FUSED_REMAP);
    a.rin = p->rec(p->buf);
    // the in-kernel remap writes L_{n+1} unless that layout is resident
    const int nbuf = p->next_buf(p->buf, (n + 1) % L.N);
    a.rout = (infuse && nbuf < 2) ? p->rec(nbuf) : nullptr;
    a.perm = p->perm(n);
    a.row_ptr = p->rp(n);
    a.shards = p->sh(n);
    a.fl = p->fl(n);
    a.order = (kind == mk::KIND_LOSS) ? nullptr : p->ord(n);
    a.rbits = p->rb(n);
    a.nrows = p->nr(n);
    a.nblk = (int32_t)L.nblk;
    a.nshards = (int32_t)p->nshards[n];
    a.mode = n;
    a.R = L.R;
    a.cw = L.cw;
    for (int w = 0; w < L.N; ++w) {
        a.fac[w] = facs[w];
        a.coff[w] = L.loff[n][w];
        a.ooff[w] = L.loff[(n + 1) % L.N][w];
        a.cmask[w] = L.cmask[w];
    }
    a.out = out;
    const int cs = p->carry_sel;
    a.carry = p->rt<float>(L.rt_carry[cs]);
    a.gscale = gscale;
    a.partial = p->rt<double>(L.rt_partial);
    const mk::LaneCfg c = lane_cfg(L.R, fdt, facs, L.N, out);
    // measurement plans: the MTTKRP kernel's loads only (contiguous lanes)
    const bool gonly = kind == mk::KIND_MTTKRP && (L.flags & MTTKRP_GATHER_ONLY);
    if (gonly && c.strided)
        return fail(p, MTTKRP_EINVAL, "MTTKRP_GATHER_ONLY needs R a multiple of 4 (FP32) or 8 "
                                      "(BF16) and 16-byte aligned factors");
    const int wpb = mk::MTT_WAVES;   // shards (waves) per workgroup
    const unsigned grid = (unsigned)((p->nshards[n] + wpb - 1) / wpb);
    const int pk = kind == mk::KIND_MTTKRP                                    ? MTTKRP_PROF_MTTKRP
                   : (kind == mk::KIND_RESID || kind == mk::KIND_RESID_LOSS) ? MTTKRP_PROF_RESID
                                            : MTTKRP_PROF_LOSS;
    ProfEvent ev{nullptr, nullptr, n, pk};
    const bool prof = p->prof;
    if (prof) {
        ev.a = take_event(p);
        ev.b = take_event(p);
        if (ev.a) HIPCHK(p, hipEventRecord(ev.a, s));
    }
    const bool seg = kind != mk::KIND_LOSS && !gonly && p->npart[n] > 0;
    if (seg) {
        mttkrp_status st = ensure_aux(p);
        if (st != MTTKRP_OK) return st;
        // the reduction that last read this carry buffer must be done
        if (p->seg_pending[cs]) HIPCHK(p, hipStreamWaitEvent(s, p->ev_seg[cs], 0));
        p->seg_pending[cs] = false;
        p->carry_sel ^= 1;
    }
    HIPCHK(p, launch_mttkrp_any(L.N, a, fdt == MTTKRP_BF16, c, gonly ? mk::KIND_GATHER : kind,
                                grid, s));
    if (prof) {
        if (ev.b) HIPCHK(p, hipEventRecord(ev.b, s));
        p->events.push_back(ev);
    }
    if (seg) {
        HIPCHK(p, hipEventRecord(p->ev_fork, s));
        HIPCHK(p, hipStreamWaitEvent(p->aux, p->ev_fork, 0));
        const int RL = std::min(256, next_pow2(L.R));
        const float *src = a.carry;
        const int32_t *ids = p->split(n);
        const int32_t *keys = p->split(n) + p->npart[n];
        int64_t P = p->npart[n];
        const int B = seg_block(L.R);
        for (int lvl = 0;; ++lvl) {
            const int64_t nb = (P + B - 1) / B;
            const int last = nb == 1;
            float *nx = p->rt<float>(L.rt_seg[lvl & 1]);
            int32_t *nk = p->rt<int32_t>(L.rt_segk[lvl & 1]);
            hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, p->aux, src,
                               ids, keys, P, B, L.R, RL, out, nx, nk, last);
            HIPCHK(p, hipGetLastError());
            if (last) break;
            src = nx;
            keys = nk;
            ids = nullptr;
            P = 2 * nb;
        }
        HIPCHK(p, hipEventRecord(p->ev_seg[cs], p->aux));
        p->seg_pending[cs] = true;
        p->seg_out[cs] = reinterpret_cast<const char *>(out);
        p->seg_out_bytes[cs] = (size_t)rows * L.R * sizeof(float);
        p->aux_pending = true;
    }
    if (infuse) {
        p->buf = nbuf;
        p->cur = (n + 1) % L.N;
    } else if (fuse) {
        return remap_step(p, s);
    }
    return MTTKRP_OK;
}

// Locality order (MTTKRP_LOCALITY_ORDER; Sec. V-J, Z-Morton ordering at
// preprocessing): out = input positions in L_n order, L_n keyed by (c_n,
// Morton(c_{n-1}, c_{n-2}), c_{n-3}, ..., c_{n+1}, input position); with two
// modes (c_n, c_{n-1}, position).  Stable LSD radix passes, least
// significant key first; the Morton code in 31-bit slices.
static mttkrp_status sort_locality(mttkrp_plan_t p, const int32_t *d_idx, int n, int32_t *out,
                                   hipStream_t s)
{
    const Layout &L = p->L;
    const int N = L.N;
    const int64_t nnz = L.nnz;
    int32_t *kb[2] = {p->rt<int32_t>(L.ps_k0), p->rt<int32_t>(L.ps_k1)};
    int32_t *vb[2] = {p->rt<int32_t>(L.ps_v0), p->rt<int32_t>(L.ps_v1)};
    const unsigned gg = grid_for(nnz);
    const int32_t *src = nullptr;
    // one stable pass over the keys the launch wrote into (kb[0], vb[0])
    auto pass = [&](int bits) -> mttkrp_status {
        HIPCHK(p, hipGetLastError());
        int which = 0;
        mttkrp_status st = radix_sort(p, kb[0], vb[0], kb[1], vb[1], nnz, bits, s, &which);
        if (st != MTTKRP_OK) return st;
        HIPCHK(p, hipMemcpyAsync(out, vb[which], nnz * 4, hipMemcpyDeviceToDevice, s));
        src = out;
        return MTTKRP_OK;
    };
    auto coord_pass = [&](int w) -> mttkrp_status {
        hipLaunchKernelGGL(plan::gather_keys_kernel, dim3(gg), dim3(256), 0, s, d_idx + w * nnz,
                           src, nnz, kb[0], vb[0], 0);
        return pass(key_bits(L.dims[w]));
    };
    mttkrp_status st;
    if (N == 2) {
        if ((st = coord_pass((n + 1) % N)) != MTTKRP_OK) return st;
    } else {
        for (int k = N - 1; k >= 3; --k)               // c_{n+1}, ..., c_{n-3}
            if ((st = coord_pass((n + N - k) % N)) != MTTKRP_OK) return st;
        const int m1 = (n + N - 1) % N, m2 = (n + N - 2) % N;
        const int zb = 2 * std::max(key_bits(L.dims[m1]), key_bits(L.dims[m2]));
        for (int shift = 0; shift < std::max(zb, 1); shift += 31) {
            hipLaunchKernelGGL(plan::morton_keys_kernel, dim3(gg), dim3(256), 0, s,
                               d_idx + m1 * nnz, d_idx + m2 * nnz, src, nnz, shift, kb[0], vb[0]);
            if ((st = pass(std::min(31, zb - shift))) != MTTKRP_OK) return st;
        }
    }
    return coord_pass(n);                              // c_n, most significant
}

// Plan steps 2-3 under the locality order: L_0's records, and per mode the
// row pointers of L_n and P_n[i] = slot in L_{n+1} of the element at slot i
// of L_n (composed from the two orders).
static mttkrp_status plan_locality(mttkrp_plan_t p, const int32_t *d_idx, const float *d_vals,
                                   hipStream_t s)
{
    const Layout &L = p->L;
    const int N = L.N;
    const int64_t nnz = L.nnz;
    int32_t *kb[2] = {p->rt<int32_t>(L.ps_k0), p->rt<int32_t>(L.ps_k1)};
    int32_t *vb1 = p->rt<int32_t>(L.ps_v1);
    int32_t *ob[2] = {p->rt<int32_t>(L.ps_o0), p->rt<int32_t>(L.ps_o1)};
    const unsigned gg = grid_for(nnz);
    mttkrp_status st = sort_locality(p, d_idx, 0, ob[0], s);
    if (st != MTTKRP_OK) return st;
    HIPCHK(p, launch_pack_any(L, d_idx, d_vals, ob[0], p->rec(0), s));
    int oc = 0;
    for (int n = 0; n < N; ++n) {
        const int nx = (n + 1) % N;
        // c_n in layout order -> row pointers of L_n
        hipLaunchKernelGGL(plan::gather_keys_kernel, dim3(gg), dim3(256), 0, s, d_idx + n * nnz,
                           ob[oc], nnz, kb[1], vb1, 1);
        hipLaunchKernelGGL(plan::row_ptr_kernel, dim3(grid_for(L.dims[n] + 1)), dim3(256), 0, s,
                           kb[1], nnz, (int32_t)L.dims[n], p->rp(n));
        HIPCHK(p, hipGetLastError());
        if ((st = sort_locality(p, d_idx, nx, ob[oc ^ 1], s)) != MTTKRP_OK) return st;
        hipLaunchKernelGGL(plan::slot_of_kernel, dim3(gg), dim3(256), 0, s, ob[oc ^ 1], nnz,
                           kb[0]);
        hipLaunchKernelGGL(plan::compose_kernel, dim3(gg), dim3(256), 0, s, kb[0], ob[oc], nnz,
                           p->perm(n));
        HIPCHK(p, hipGetLastError());
        oc ^= 1;
    }
    return MTTKRP_OK;
}

// ---------------------------------------------------------------- C ABI
extern "C" {

const char *mttkrp_status_str(mttkrp_status st)
{
    switch (raw_enum(st)) {
    case MTTKRP_OK: return "ok";
    case MTTKRP_EINVAL: return "invalid argument";
    case MTTKRP_ERANGE: return "coordinate out of range";
    case MTTKRP_ENOMEM: return "workspace too small";
    case MTTKRP_ESTATE: return "tensor is in another mode's layout";
    case MTTKRP_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *mttkrp_last_error(mttkrp_plan_t p)
{
    return p ? p->err.c_str() : g_last_error.c_str();
}

mttkrp_status mttkrp_plan_workspace(int nmodes, const int64_t *dims, int64_t nnz, int rank,
                                    const mttkrp_plan_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(nullptr, MTTKRP_EINVAL, "bytes is NULL");
    Layout L;
    std::string why;
    mttkrp_status st = compute_layout(nmodes, dims, nnz, rank, opts, &L, &why);
    if (st != MTTKRP_OK) return fail(nullptr, st, why);
    *bytes = L.total;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_plan(int nmodes, const int64_t *dims, int64_t nnz, const int32_t *d_idx,
                          const float *d_vals, int rank, const mttkrp_plan_opts *opts,
                          void *d_workspace, size_t ws_bytes, void *stream, mttkrp_plan_t *out)
{
    if (!out) return fail(nullptr, MTTKRP_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    std::string why;
    mttkrp_status st = compute_layout(nmodes, dims, nnz, rank, opts, &L, &why);
    if (st != MTTKRP_OK) return fail(nullptr, st, why);
    if (!d_workspace) return fail(nullptr, MTTKRP_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
        return fail(nullptr, MTTKRP_EINVAL, "workspace must be 256-byte aligned");
    if (nnz > 0 && (!d_idx || !d_vals)) return fail(nullptr, MTTKRP_EINVAL, "idx/vals is NULL");
    if (ws_bytes < L.total)
        return fail(nullptr, MTTKRP_ENOMEM,
                    "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                        std::to_string(L.total));
    mttkrp_plan_t p = new (std::nothrow) mttkrp_plan_s();
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "host allocation failed");
    p->L = L;
    p->ws = reinterpret_cast<char *>(d_workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int N = L.N;
    auto bail = [&](mttkrp_status e) {
        g_last_error = p->err;
        delete p;
        return e;
    };
    if (nnz == 0) {
        for (int n = 0; n < N; ++n) {
            if (hipMemsetAsync(p->rp(n), 0, (L.dims[n] + 1) * 4, s) != hipSuccess)
                return bail(fail(p, MTTKRP_EHIP, "hipMemsetAsync failed"));
            p->nempty[n] = L.dims[n];
        }
        if (hipMemsetAsync(p->xx(), 0, 8, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(p, MTTKRP_EHIP, "initialisation failed"));
        *out = p;
        return MTTKRP_OK;
    }
    // 1. index validation
    int32_t *err = p->rt<int32_t>(L.ps_err);
    plan::Dims8 d8;
    for (int n = 0; n < 8; ++n) d8.d[n] = n < N ? (int32_t)L.dims[n] : 0;
    int32_t herr = 0;
    if (hipMemsetAsync(err, 0, 4, s) != hipSuccess) return bail(fail(p, MTTKRP_EHIP, "memset"));
    hipLaunchKernelGGL(plan::validate_kernel, dim3(grid_for(nnz * N)), dim3(256), 0, s, d_idx, N,
                       nnz, d8, err);
    if (hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(p, MTTKRP_EHIP, std::string("validation: ") +
                                             hipGetErrorString(hipGetLastError())));
    if (herr) return bail(fail(p, MTTKRP_ERANGE, "a coordinate is outside [0, I_n)"));

    int32_t *kb[2] = {p->rt<int32_t>(L.ps_k0), p->rt<int32_t>(L.ps_k1)};
    int32_t *vb[2] = {p->rt<int32_t>(L.ps_v0), p->rt<int32_t>(L.ps_v1)};
    int32_t *ob[2] = {p->rt<int32_t>(L.ps_o0), p->rt<int32_t>(L.ps_o1)};
    const unsigned gg = grid_for(nnz);
    if (L.flags & MTTKRP_LOCALITY_ORDER) {
        st = plan_locality(p, d_idx, d_vals, s);
        if (st != MTTKRP_OK) return bail(st);
    } else {
    // 2. L_0: stable LSD sort of input positions by c_1, c_2, ..., c_{N-1}, c_0
    const int32_t *src = nullptr;
    for (int t = 1; t <= N; ++t) {
        const int w = t % N;
        hipLaunchKernelGGL(plan::gather_keys_kernel, dim3(gg), dim3(256), 0, s, d_idx + w * nnz,
                           src, nnz, kb[0], vb[0], 0);
        int which = 0;
        st = radix_sort(p, kb[0], vb[0], kb[1], vb[1], nnz, key_bits(L.dims[w]), s, &which);
        if (st != MTTKRP_OK) return bail(st);
        // keep the permutation in ob[0]
        if (hipMemcpyAsync(ob[0], vb[which], nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return bail(fail(p, MTTKRP_EHIP, "copy"));
        src = ob[0];
    }
    if (launch_pack_any(L, d_idx, d_vals, ob[0], p->rec(0), s) != hipSuccess)
        return bail(fail(p, MTTKRP_EHIP, "pack launch"));
    // 3. per mode: row pointers of L_n; P_n by a stable sort of L_n by c_{n+1}
    int oc = 0;
    for (int n = 0; n < N; ++n) {
        const int nx = (n + 1) % N;
        // c_n in layout order (sorted) into kb[1], free until the sort below
        hipLaunchKernelGGL(plan::gather_keys_kernel, dim3(gg), dim3(256), 0, s, d_idx + n * nnz,
                           ob[oc], nnz, kb[1], vb[1], 1);
        hipLaunchKernelGGL(plan::row_ptr_kernel, dim3(grid_for(L.dims[n] + 1)), dim3(256), 0, s,
                           kb[1], nnz, (int32_t)L.dims[n], p->rp(n));
        hipLaunchKernelGGL(plan::gather_keys_kernel, dim3(gg), dim3(256), 0, s, d_idx + nx * nnz,
                           ob[oc], nnz, kb[0], vb[0], 1);
        int which = 0;
        st = radix_sort(p, kb[0], vb[0], kb[1], vb[1], nnz, key_bits(L.dims[nx]), s, &which);
        if (st != MTTKRP_OK) return bail(st);
        hipLaunchKernelGGL(plan::invert_kernel, dim3(gg), dim3(256), 0, s, vb[which], nnz,
                           p->perm(n), ob[oc], ob[oc ^ 1]);
        if (hipGetLastError() != hipSuccess) return bail(fail(p, MTTKRP_EHIP, "plan kernels"));
        oc ^= 1;
    }
    }
    // ||X||^2 for the fit
    {
        const int nb = 1024;
        double *part = p->rt<double>(L.rt_partial);   // sort buffers are free now
        if (hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(p, MTTKRP_EHIP, "plan sync"));
        hipLaunchKernelGGL(als::sumsq_partial, dim3(nb), dim3(256), 0, s, p->rec(0), nnz,
                           L.cw + 1, part);
        hipLaunchKernelGGL(als::sum_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)nb, p->xx());
    }
    // 4. host partition tables, row-start tables
    std::vector<int32_t> rp, shards, order, split, bins, fl, nrows, rids;
    std::vector<uint32_t> rtab;
    for (int n = 0; n < N; ++n) {
        rp.resize(L.dims[n] + 1);
        if (hipMemcpyAsync(rp.data(), p->rp(n), rp.size() * 4, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(p, MTTKRP_EHIP, "row pointer copy"));
        build_tables(L, n, rp, shards, order, split, bins, fl, &p->nempty[n], &p->nsplit[n]);
        build_row_starts(L, n, rp, rtab, nrows, rids);
        p->nshards[n] = (int64_t)shards.size() / 3;
        p->npart[n] = (int64_t)split.size() / 2;
        if (p->nshards[n] > L.maxS[n]) return bail(fail(p, MTTKRP_EINVAL, "shard bound"));
        if (hipMemcpyAsync(p->sh(n), shards.data(), shards.size() * 4, hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            hipMemcpyAsync(p->fl(n), fl.data(), fl.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(p->rb(n), rtab.data(), rtab.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(p->nr(n), nrows.data(), nrows.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(p->rid(n), rids.data(), rids.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(p->ord(n), order.data(), order.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            (!split.empty() && hipMemcpyAsync(p->split(n), split.data(), split.size() * 4,
                                              hipMemcpyHostToDevice, s) != hipSuccess) ||
            hipMemcpyAsync(p->lpt(n), bins.data(), bins.size() * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(p, MTTKRP_EHIP, "table upload"));
    }
    // resident layouts: one sweep of remaps through the work buffers (which
    // needs the row-start tables above), each resident layout copied out as
    // it is reached; L_0 ends in work buffer N mod 2 (or is read from its
    // resident copy)
    int buf0 = 0;
    if (L.resident) {
        const size_t rbytes = (size_t)nnz * (L.cw + 1) * 4;
        int b = 0;
        for (int n = 0; n < N; ++n) {
            if ((L.resident >> n & 1u) &&
                hipMemcpyAsync(p->rec(2 + n), p->rec(b), rbytes, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                return bail(fail(p, MTTKRP_EHIP, "resident layout copy"));
            if (launch_remap_any(p, n, p->rec(b), p->rec(b ^ 1), s) != hipSuccess)
                return bail(fail(p, MTTKRP_EHIP, "resident layout remap"));
            b ^= 1;
        }
        buf0 = (L.resident & 1u) ? 2 : b;
    }
    if (hipMemsetAsync(p->ridge(), 0, 8, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(p, MTTKRP_EHIP, "plan finish"));
    // the side stream and its events exist from here on, so that no later
    // call creates HIP objects
    if (ensure_aux(p) != MTTKRP_OK) {
        g_last_error = p->err;
        mttkrp_plan_destroy(p);
        return MTTKRP_EHIP;
    }
    p->cur = 0;
    p->buf = buf0;
    *out = p;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_plan_destroy(mttkrp_plan_t p)
{
    if (!p) return MTTKRP_EINVAL;
    for (auto &e : p->events) {
        if (e.a) (void)hipEventDestroy(e.a);
        if (e.b) (void)hipEventDestroy(e.b);
    }
    for (auto e : p->pool) (void)hipEventDestroy(e);
    if (p->aux) {
        (void)hipStreamSynchronize(p->aux);
        (void)hipStreamDestroy(p->aux);
        for (hipEvent_t e : {p->ev_fork, p->ev_join, p->ev_seg[0], p->ev_seg[1], p->ev_als})
            if (e) (void)hipEventDestroy(e);
    }
    delete p;
    return MTTKRP_OK;
}

mttkrp_status remap(mttkrp_plan_t p, int to_mode, void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    if (to_mode < 0 || to_mode >= p->L.N) return fail(p, MTTKRP_EINVAL, "bad mode");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    while (p->cur != to_mode) {
        mttkrp_status st = remap_step(p, s);
        if (st != MTTKRP_OK) return st;
    }
    return MTTKRP_OK;
}

static mttkrp_status reach(mttkrp_plan_t p, int mode, hipStream_t s)
{
    if (p->cur == mode) return MTTKRP_OK;
    if (p->L.flags & MTTKRP_NO_IMPLICIT_REMAP)
        return fail(p, MTTKRP_ESTATE,
                    "tensor is in layout " + std::to_string(p->cur) + ", not " +
                        std::to_string(mode));
    while (p->cur != mode) {
        mttkrp_status st = remap_step(p, s);
        if (st != MTTKRP_OK) return st;
    }
    return MTTKRP_OK;
}

mttkrp_status mttkrp_mode(mttkrp_plan_t p, int mode, const void *const *d_factors,
                          mttkrp_dtype fdt, float *d_out, int fuse_remap, void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    if (mode < 0 || mode >= p->L.N) return fail(p, MTTKRP_EINVAL, "bad mode");
    if (!d_out) return fail(p, MTTKRP_EINVAL, "out is NULL");
    mttkrp_status st = check_factors(p, d_factors, 1, mode, fdt);
    if (st != MTTKRP_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = reach(p, mode, s);
    if (st != MTTKRP_OK) return st;
    st = run_pass(p, d_factors, fdt, d_out, fuse_remap != 0, mk::KIND_MTTKRP, nullptr, s);
    if (st != MTTKRP_OK) return st;
    return join_aux(p, s);
}

mttkrp_status mttkrp_all_modes(mttkrp_plan_t p, const void *const *d_factors, mttkrp_dtype fdt,
                               float *const *d_out, void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    if (!d_out) return fail(p, MTTKRP_EINVAL, "out is NULL");
    for (int n = 0; n < p->L.N; ++n)
        if (!d_out[n]) return fail(p, MTTKRP_EINVAL, "out pointer is NULL");
    mttkrp_status st = check_factors(p, d_factors, 0, -1, fdt);
    if (st != MTTKRP_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t saved = p->L.flags;
    p->L.flags &= ~MTTKRP_NO_IMPLICIT_REMAP;
    st = reach(p, 0, s);
    p->L.flags = saved;
    if (st != MTTKRP_OK) return st;
    for (int n = 0; n < p->L.N; ++n) {
        st = run_pass(p, d_factors, fdt, d_out[n], true, mk::KIND_MTTKRP, nullptr, s);
        if (st != MTTKRP_OK) return st;
    }
    return join_aux(p, s);
}

mttkrp_status cp_loss_grad(mttkrp_plan_t p, const void *const *d_factors, mttkrp_dtype fdt,
                           double *d_loss, float *const *d_grads, const double *d_grad_scale,
                           void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    mttkrp_status st = check_factors(p, d_factors, 0, -1, fdt);
    if (st != MTTKRP_OK) return st;
    if (d_grads)
        for (int k = 0; k < p->L.N; ++k)
            if (!d_grads[k]) return fail(p, MTTKRP_EINVAL, "gradient pointer is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Layout &L = p->L;
    // loss and gradients: the first residual pass also sums the squared
    // residuals (identical terms, order and partials as the loss pass), so
    // the loss costs no pass of its own; the in-kernel remap form keeps the
    // separate loss pass
    const bool joint = d_loss && d_grads && L.nnz > 0 && !(L.flags & MTTKRP_FUSED_REMAP);
    if (d_loss && !joint) {
        if (L.nnz == 0) {
            HIPCHK(p, hipMemsetAsync(d_loss, 0, 8, s));
        } else {
            st = run_pass(p, d_factors, fdt, nullptr, false, mk::KIND_LOSS, nullptr, s);
            if (st != MTTKRP_OK) return st;
            hipLaunchKernelGGL(als::sum_kernel, dim3(1), dim3(256), 0, s,
                               p->rt<double>(L.rt_partial), p->nshards[p->cur], d_loss);
            HIPCHK(p, hipGetLastError());
        }
    }
    if (d_grads) {
        const int start = p->cur;
        for (int t = 0; t < L.N; ++t) {
            const int k = (start + t) % L.N;
            const bool with_loss = joint && t == 0;
            st = run_pass(p, d_factors, fdt, d_grads[k], true,
                          with_loss ? mk::KIND_RESID_LOSS : mk::KIND_RESID, d_grad_scale, s);
            if (st != MTTKRP_OK) return st;
            if (with_loss) {
                // the partials of mode k's shards; the remap that followed
                // does not touch them
                hipLaunchKernelGGL(als::sum_kernel, dim3(1), dim3(256), 0, s,
                                   p->rt<double>(L.rt_partial), p->nshards[k], d_loss);
                HIPCHK(p, hipGetLastError());
            }
        }
    }
    return join_aux(p, s);
}

// One Gauss-Seidel sweep.  grams_valid: the Gram matrices of every mode are
// those of the current stored factors (the previous sweep of the same
// driver call left them so), and are not recomputed.
static mttkrp_status als_sweep(mttkrp_plan_t p, void *const *d_factors, mttkrp_dtype fdt,
                               float *d_mbuf, double *d_lambda, double *d_fit, bool grams_valid,
                               hipStream_t s)
{
    mttkrp_status st;
    const Layout &L = p->L;
    const int N = L.N, R = L.R;
    const bool bf = fdt == MTTKRP_BF16;
    double *G = p->rt<double>(L.rt_G);
    double *gpart = p->rt<double>(L.rt_gpart);
    const int tiles = (R + als::GRAM_TILE - 1) / als::GRAM_TILE;
    const int gbmax = std::max(1, GRAM_TARGET_BLOCKS / (tiles * tiles));
    auto gram = [&](int w, hipStream_t gs) -> mttkrp_status {
        const int64_t I = L.dims[w];
        // at least 256 rows per block
        const int gb = (int)std::max<int64_t>(1, std::min<int64_t>(gbmax, (I + 255) / 256));
        const int64_t chunk = (I + gb - 1) / gb;
        const dim3 grid(gb, tiles, tiles), blk(256);
        if (bf)
            hipLaunchKernelGGL(als::gram_partial<uint16_t>, grid, blk, 0, gs,
                               (const uint16_t *)d_factors[w], I, R, chunk, gpart);
        else
            hipLaunchKernelGGL(als::gram_partial<float>, grid, blk, 0, gs,
                               (const float *)d_factors[w], I, R, chunk, gpart);
        hipLaunchKernelGGL(als::gram_reduce, dim3(R * R), dim3(64), 0, gs, gpart, gb, R,
                           G + (int64_t)w * R * R);
        HIPCHK(p, hipGetLastError());
        return MTTKRP_OK;
    };
    const uint32_t saved = p->L.flags;
    p->L.flags &= ~MTTKRP_NO_IMPLICIT_REMAP;
    st = reach(p, 0, s);
    p->L.flags = saved;
    if (st != MTTKRP_OK) return st;
    if (!grams_valid)
        for (int w = 0; w < N; ++w)
            if ((st = gram(w, s)) != MTTKRP_OK) return st;
    const int RT = std::min(256, next_pow2(R));
    double *colsq = p->rt<double>(L.rt_colsq);
    // The update of A_n needs M_n (the MTTKRP and the split-row reduction on
    // the side stream) but not the remap that follows the MTTKRP, and the
    // remap needs nothing from the update.  So the update runs on the side
    // stream, after the reduction, while the remap runs on `s`; the next
    // MTTKRP, which reads A_n and overwrites M_n, waits for both.  (With the
    // remap inside the MTTKRP kernel there is nothing to overlap: everything
    // stays on `s`.)  Each kernel does the same work in the same order
    // either way, so the results are identical.
    const bool overlap = !(L.flags & MTTKRP_FUSED_REMAP);
    hipStream_t as = overlap ? p->aux : s;
    for (int n = 0; n < N; ++n) {
        if ((st = join_aux(p, s)) != MTTKRP_OK) return st;      // A_{n-1} stored
        st = run_pass(p, (const void *const *)d_factors, fdt, d_mbuf, !overlap,
                      mk::KIND_MTTKRP, nullptr, s);
        if (st != MTTKRP_OK) return st;
        if (overlap) {
            // the side stream: after this MTTKRP (and, in stream order, after
            // its split-row reduction) -> M_n complete there
            HIPCHK(p, hipEventRecord(p->ev_als, s));
            HIPCHK(p, hipStreamWaitEvent(p->aux, p->ev_als, 0));
        } else if ((st = join_aux(p, s)) != MTTKRP_OK) {
            return st;                                          // M_n complete on s
        }
        hipLaunchKernelGGL(als::chol_inverse, dim3(1), dim3(256), 0, as, G, N, n, R,
                           p->rt<double>(L.rt_L), p->rt<double>(L.rt_Linv), p->rt<double>(L.rt_W),
                           p->ridge(), p->fail());
        const int64_t I = L.dims[n];
        const double *W = p->rt<double>(L.rt_W);
        if (bf) {
            hipLaunchKernelGGL(als::als_apply<uint16_t>, dim3(als::APPLY_BLOCKS), dim3(256), 0, as,
                               d_mbuf, I, R, RT, W, 0, colsq, d_lambda, (uint16_t *)d_factors[n]);
            hipLaunchKernelGGL(als::lambda_kernel, dim3(R), dim3(256), 0, as, colsq,
                               als::APPLY_BLOCKS, R, d_lambda);
            hipLaunchKernelGGL(als::als_apply<uint16_t>, dim3(als::APPLY_BLOCKS), dim3(256), 0, as,
                               d_mbuf, I, R, RT, W, 1, colsq, d_lambda, (uint16_t *)d_factors[n]);
        } else {
            hipLaunchKernelGGL(als::als_apply<float>, dim3(als::APPLY_BLOCKS), dim3(256), 0, as,
                               d_mbuf, I, R, RT, W, 0, colsq, d_lambda, (float *)d_factors[n]);
            hipLaunchKernelGGL(als::lambda_kernel, dim3(R), dim3(256), 0, as, colsq,
                               als::APPLY_BLOCKS, R, d_lambda);
            hipLaunchKernelGGL(als::als_apply<float>, dim3(als::APPLY_BLOCKS), dim3(256), 0, as,
                               d_mbuf, I, R, RT, W, 1, colsq, d_lambda, (float *)d_factors[n]);
        }
        HIPCHK(p, hipGetLastError());
        if ((st = gram(n, as)) != MTTKRP_OK) return st;
        if (overlap) {
            p->aux_pending = true;
            if ((st = remap_step(p, s)) != MTTKRP_OK) return st;   // beside the update
        }
    }
    // everything the side stream did is complete on `s` when the call's work
    // is (the fit below reads M_{N-1} and A_{N-1})
    if ((st = join_aux(p, s)) != MTTKRP_OK) return st;
    if (d_fit) {
        const int n = N - 1;
        double *inner = colsq;
        if (bf)
            hipLaunchKernelGGL(als::inner_partial<uint16_t>, dim3(als::APPLY_BLOCKS), dim3(256), 0,
                               s, d_mbuf, (const uint16_t *)d_factors[n], L.dims[n], R, RT, inner);
        else
            hipLaunchKernelGGL(als::inner_partial<float>, dim3(als::APPLY_BLOCKS), dim3(256), 0, s,
                               d_mbuf, (const float *)d_factors[n], L.dims[n], R, RT, inner);
        hipLaunchKernelGGL(als::fit_kernel, dim3(1), dim3(256), 0, s, inner, als::APPLY_BLOCKS, G,
                           N, d_lambda, R, p->xx(), d_fit);
        HIPCHK(p, hipGetLastError());
    }
    return MTTKRP_OK;
}

static mttkrp_status als_args(mttkrp_plan_t p, void *const *d_factors, const mttkrp_dtype &fdt,
                              float *d_mbuf, double *d_lambda)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    mttkrp_status st = check_factors(p, (const void *const *)d_factors, 0, -1, fdt);
    if (st != MTTKRP_OK) return st;
    if (!d_mbuf || !d_lambda) return fail(p, MTTKRP_EINVAL, "mbuf/lambda is NULL");
    return MTTKRP_OK;
}

mttkrp_status cp_als_sweep(mttkrp_plan_t p, void *const *d_factors, mttkrp_dtype fdt,
                           float *d_mbuf, double *d_lambda, double *d_fit, void *stream)
{
    mttkrp_status st = als_args(p, d_factors, fdt, d_mbuf, d_lambda);
    if (st != MTTKRP_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(als::zero_i32, dim3(1), dim3(64), 0, s, p->ridge(), 2);
    HIPCHK(p, hipGetLastError());
    return als_sweep(p, d_factors, fdt, d_mbuf, d_lambda, d_fit, false, s);
}

}  // extern "C"

// Scratch of cp_als_sweep_static: the MTTKRP output M_n of the sweep, one
// array per GPU (each device holds its own copy of the module's globals),
// kept until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device below.
static __device__ __align__(256) float scratch[MTTKRP_STATIC_MBUF_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
mttkrp_status static_scratch(mttkrp_plan_t p, float **out)
{
    int dev = -1;
    HIPCHK(p, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(p, MTTKRP_EINVAL, "device ordinal beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(p, MTTKRP_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e));
        g_scratch[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch[dev];
    return MTTKRP_OK;
}
}  // namespace

extern "C" {

mttkrp_status cp_als_sweep_static(mttkrp_plan_t p, void *const *d_factors, mttkrp_dtype fdt,
                                  double *d_lambda, double *d_fit, void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    int64_t need = 0;
    for (int n = 0; n < p->L.N; ++n) need = std::max<int64_t>(need, p->L.dims[n] * p->L.R);
    if (need > MTTKRP_STATIC_MBUF_FLOATS)
        return fail(p, MTTKRP_EINVAL,
                    "max_n I_n * R = " + std::to_string((long long)need) +
                        " exceeds the static scratch of " +
                        std::to_string((long long)MTTKRP_STATIC_MBUF_FLOATS) +
                        " floats; use cp_als_sweep with a caller buffer");
    float *mbuf = nullptr;
    mttkrp_status st = static_scratch(p, &mbuf);
    if (st != MTTKRP_OK) return st;
    st = als_args(p, d_factors, fdt, mbuf, d_lambda);
    if (st != MTTKRP_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // kernel timing would create HIP events: suspended for this call
    const bool prof = p->prof;
    p->prof = false;
    hipLaunchKernelGGL(als::zero_i32, dim3(1), dim3(64), 0, s, p->ridge(), 2);
    st = hipGetLastError() == hipSuccess ? MTTKRP_OK : fail(p, MTTKRP_EHIP, "launch");
    if (st == MTTKRP_OK) st = als_sweep(p, d_factors, fdt, mbuf, d_lambda, d_fit, false, s);
    p->prof = prof;
    return st;
}

mttkrp_status cp_als(mttkrp_plan_t p, void *const *d_factors, mttkrp_dtype fdt, float *d_mbuf,
                     double *d_lambda, int max_sweeps, double tol, double *d_fit_trace,
                     int *sweeps, double *fit, void *stream)
{
    mttkrp_status st = als_args(p, d_factors, fdt, d_mbuf, d_lambda);
    if (st != MTTKRP_OK) return st;
    if (max_sweeps < 1) return fail(p, MTTKRP_EINVAL, "max_sweeps must be >= 1");
    if (!(tol >= 0.0)) return fail(p, MTTKRP_EINVAL, "tol must be >= 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(als::zero_i32, dim3(1), dim3(64), 0, s, p->ridge(), 2);
    HIPCHK(p, hipGetLastError());
    double prev = 0.0, cur = 0.0;
    int k = 0;
    while (k < max_sweeps) {
        double *slot = d_fit_trace ? d_fit_trace + k : p->fit_slot();
        st = als_sweep(p, d_factors, fdt, d_mbuf, d_lambda, slot, k > 0, s);
        if (st != MTTKRP_OK) return st;
        HIPCHK(p, hipMemcpyAsync(&cur, slot, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(p, hipStreamSynchronize(s));
        ++k;
        if (k > 1 && std::fabs(cur - prev) < tol) break;
        prev = cur;
    }
    if (sweeps) *sweeps = k;
    if (fit) *fit = cur;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_plan_query(mttkrp_plan_t p, int what, int mode, void *dst, size_t bytes,
                                void *stream)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    if (mode < 0 || mode >= p->L.N) return fail(p, MTTKRP_EINVAL, "bad mode");
    int64_t need = 0;
    const Layout &L = p->L;
    const void *src = nullptr;
    switch (what) {
    case MTTKRP_Q_LAYOUT: need = L.nnz * (L.N + 1) * 4; src = p->rec(p->buf); break;
    case MTTKRP_Q_PERM: need = L.nnz * 4; src = p->perm(mode); break;
    case MTTKRP_Q_ROW_PTR: need = (L.dims[mode] + 1) * 4; src = p->rp(mode); break;
    case MTTKRP_Q_SHARDS: need = p->nshards[mode] * 12; src = p->sh(mode); break;
    case MTTKRP_Q_LPT: need = L.k[mode] * 4; src = p->lpt(mode); break;
    default: return fail(p, MTTKRP_EINVAL, "bad query");
    }
    if (!dst || bytes < (size_t)need) return fail(p, MTTKRP_EINVAL, "destination too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (what == MTTKRP_Q_LAYOUT && need > 0) {
        // stored records are bit-packed and omit the layout's own coordinate:
        // widen to N coordinates + value, that coordinate taken from the
        // row pointers, in chunks so that the host buffers stay small for
        // any nnz
        const int NW = L.cw + 1, N = L.N, m = p->cur;
        const int64_t CH = int64_t(1) << 20;
        std::vector<uint32_t> packed((size_t)std::min(CH, L.nnz) * NW);
        std::vector<uint32_t> wide((size_t)std::min(CH, L.nnz) * (N + 1));
        std::vector<int32_t> rp((size_t)L.dims[m] + 1);
        HIPCHK(p, hipMemcpyAsync(rp.data(), p->rp(m), rp.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(p, hipStreamSynchronize(s));
        int64_t row = 0;
        const uint32_t *srec = static_cast<const uint32_t *>(src);
        char *out = static_cast<char *>(dst);
        for (int64_t c0 = 0; c0 < L.nnz; c0 += CH) {
            const int64_t cn = std::min(CH, L.nnz - c0);
            HIPCHK(p, hipMemcpyAsync(packed.data(), srec + c0 * NW, (size_t)cn * NW * 4,
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(p, hipStreamSynchronize(s));
            for (int64_t i = 0; i < cn; ++i) {
                const uint32_t *r = packed.data() + i * NW;
                uint32_t *o = wide.data() + i * (N + 1);
                while (rp[row + 1] <= c0 + i) ++row;     // row holding position c0 + i
                for (int n = 0; n < N; ++n) {
                    if (n == m) {
                        o[n] = (uint32_t)row;
                        continue;
                    }
                    const uint32_t off = L.loff[m][n], q = off >> 5;
                    const uint64_t x = ((uint64_t)r[q + 1] << 32) | r[q];
                    o[n] = (uint32_t)(x >> (off & 31u)) & L.cmask[n];
                }
                o[N] = r[NW - 1];
            }
            HIPCHK(p, hipMemcpyAsync(out + c0 * (N + 1) * 4, wide.data(), (size_t)cn * (N + 1) * 4,
                                     hipMemcpyDefault, s));
            HIPCHK(p, hipStreamSynchronize(s));
        }
        return MTTKRP_OK;
    }
    if (need > 0) HIPCHK(p, hipMemcpyAsync(dst, src, need, hipMemcpyDefault, s));
    HIPCHK(p, hipStreamSynchronize(s));
    return MTTKRP_OK;
}

mttkrp_status mttkrp_plan_info(mttkrp_plan_t p, int what, int mode, int64_t *value)
{
    if (!p || !value) return fail(p, MTTKRP_EINVAL, "NULL argument");
    const Layout &L = p->L;
    auto mode_ok = [&]() { return mode >= 0 && mode < L.N; };
    switch (what) {
    case MTTKRP_INFO_CUR_MODE: *value = p->cur; return MTTKRP_OK;
    case MTTKRP_INFO_RECORD_BYTES: *value = 4 * (L.cw + 1); return MTTKRP_OK;
    case MTTKRP_INFO_G: *value = L.g; return MTTKRP_OK;
    case MTTKRP_INFO_NSHARDS:
    case MTTKRP_INFO_NSUPER:
    case MTTKRP_INFO_NSPLIT:
    case MTTKRP_INFO_M:
        if (!mode_ok()) return fail(p, MTTKRP_EINVAL, "bad mode");
        *value = what == MTTKRP_INFO_NSHARDS ? p->nshards[mode]
                 : what == MTTKRP_INFO_NSUPER ? L.k[mode]
                 : what == MTTKRP_INFO_NSPLIT ? p->nsplit[mode]
                                              : L.m[mode];
        return MTTKRP_OK;
    case MTTKRP_INFO_RIDGE: {
        int32_t h = 0;
        HIPCHK(p, hipDeviceSynchronize());
        HIPCHK(p, hipMemcpy(&h, p->ridge(), 4, hipMemcpyDeviceToHost));
        *value = h;
        return MTTKRP_OK;
    }
    }
    return fail(p, MTTKRP_EINVAL, "bad info key");
}

mttkrp_status mttkrp_profile(mttkrp_plan_t p, int enable)
{
    if (!p) return fail(nullptr, MTTKRP_EINVAL, "plan is NULL");
    p->prof = enable != 0;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_profile_read(mttkrp_plan_t p, int kernel, int mode, double *ms,
                                  int64_t *launches)
{
    if (!p || !ms || !launches) return fail(p, MTTKRP_EINVAL, "NULL argument");
    if (kernel < MTTKRP_PROF_MTTKRP || kernel > MTTKRP_PROF_LOSS)
        return fail(p, MTTKRP_EINVAL, "bad kernel id");
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &e : p->events) {
        if (e.a && e.b && e.kernel == kernel && (mode < 0 || e.mode == mode)) {
            HIPCHK(p, hipEventSynchronize(e.b));
            float t = 0.0f;
            HIPCHK(p, hipEventElapsedTime(&t, e.a, e.b));
            tot += t;
            ++cnt;
        }
    }
    std::vector<ProfEvent> keep;
    for (auto &e : p->events) {
        if (e.kernel != kernel || (mode >= 0 && e.mode != mode)) {
            keep.push_back(e);
            continue;
        }
        if (e.a) p->pool.push_back(e.a);
        if (e.b) p->pool.push_back(e.b);
    }
    p->events.swap(keep);
    *ms = tot;
    *launches = cnt;
    return MTTKRP_OK;
}

}  // extern "C"
