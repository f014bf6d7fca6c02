// Per-mode sparse MTTKRP with fused dynamic remapping, the residual
// (loss-gradient) variant, the sampled-loss forward, and the standalone
// remap, templated on the number of modes N and the factor storage type.
//
// Work decomposition.  The tensor buffer holds layout L_n: nonzeros
// contiguous by output row c_n (Sec. III-B).  The plan cuts it into shards
// of at most g nonzeros that never cross a super-shard (Sec. III-A); one
// wave64 processes one shard.  Lanes run along the rank: a nonzero is
// handled by LANES lanes holding V consecutive ranks each (16-byte factor
// gathers), so one step covers SW = 64/LANES consecutive nonzeros.
//
// Per nonzero (elementwise update, Sec. II-C / Eq. 4): gather the N-1 input
// factor rows, form their Hadamard product in registers, scale by the
// value.  Rows are reduced with a segmented inclusive scan across the SW
// slots of a step plus a running carry across steps, so every output row is
// produced by one wave in a fixed order: rows wholly inside the shard are
// written directly, the shard's first row (if it began in an earlier shard)
// and last row (if it continues) go to a per-shard partial slot that the
// carry fix-up kernel adds in shard order.  No global atomics anywhere
// (lock-free ownership of output rows, Sec. IV).
//
// Remap (Alg. "Dynasor", store into the next mode's shard): lane 0 of each
// slot copies the whole record to L_{n+1}[P_n[e]], the slot precomputed by
// the plan, in the same pass (Sec. V-B: same agent).
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
            int r = sub + 64 * j;
            x[j] = (r < R) ? p[r] : 0.0f;
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
            int r = sub + 64 * j;
            x[j] = (r < R) ? bf16_to_f32(p[r]) : 0.0f;
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

// Product of the factor rows of every mode except `skip` (skip = -1: all).
template <int N, typename FT, int V, bool STRIDED>
__device__ __forceinline__ void row_product(const Args &a, const Rec<N> &rc, int skip, int sub,
                                            float (&pr)[V])
{
#pragma unroll
    for (int j = 0; j < V; ++j) pr[j] = 1.0f;
#pragma unroll
    for (int w = 0; w < N; ++w) {
        if (w == skip) continue;
        float x[V];
        Fetch<FT, V, STRIDED>::get(a.fac[w], (int64_t)rc.w[w], a.R, sub, x);
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

// ---- per-mode MTTKRP (RESID = false) / loss-gradient pass (RESID = true) --
template <int N, typename FT, int LANES, int V, bool STRIDED, bool RESID>
__global__ __launch_bounds__(256) void mttkrp_kernel(Args a)
{
    constexpr int SW = WAVE / LANES;
    const int lane = threadIdx.x & 63;
    const int sidx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sidx >= a.nshards) return;                         // whole wave
    const int shard = a.order ? a.order[sidx] : sidx;
    const int start = a.shards[3 * shard];
    const int end = start + a.shards[3 * shard + 1];
    const int n = a.mode, R = a.R;
    const int slot = lane / LANES, sub = lane % LANES;
    const bool ract = lane_active<LANES, V, STRIDED>(sub, R);
    const int f = (int)a.rin[(int64_t)start * (N + 1) + n];
    const int l = (int)a.rin[(int64_t)(end - 1) * (N + 1) + n];
    const bool split_before = a.row_ptr[f] < start;
    float coef = 1.0f;
    if constexpr (RESID) coef = -2.0f * (a.gscale ? (float)a.gscale[0] : 1.0f);
    float *const cbase = a.carry + (int64_t)shard * 2 * R;

    // flush of a row that is complete inside this shard or is its first row
    auto flush_mid = [&](int row, const float (&v)[V]) {
        float *dst = (row == f && split_before) ? cbase : a.out + (int64_t)row * R;
        store_row<V, STRIDED>(dst, R, sub, v);
    };

    float carry[V];
#pragma unroll
    for (int j = 0; j < V; ++j) carry[j] = 0.0f;
    int carry_row = -1;

    for (int base = start; base < end; base += SW) {
        const int e = base + slot;
        const bool valid = e < end;
        float p[V], pr[V];
        int row = l;                       // invalid tail slots join row l
        float val = 0.0f, m = 0.0f;
#pragma unroll
        for (int j = 0; j < V; ++j) { p[j] = 0.0f; pr[j] = 0.0f; }
        if (valid) {
            const Rec<N> rc = load_rec<N>(a.rin, e);
            row = (int)rc.w[n];
            if (a.rout && sub == 0) store_rec<N>(a.rout, a.perm[e], rc);
            if (ract) {
                val = __uint_as_float(rc.w[N]);
                row_product<N, FT, V, STRIDED>(a, rc, n, sub, pr);
                if constexpr (RESID) {
                    float xn[V];
                    Fetch<FT, V, STRIDED>::get(a.fac[n], (int64_t)row, R, sub, xn);
#pragma unroll
                    for (int j = 0; j < V; ++j) m += pr[j] * xn[j];
                }
            }
        }
        if constexpr (RESID) {
            // model value m_e: lanes outside the rank range hold 0
            m = slot_sum<LANES>(m);
            const float c = coef * (val - m);
#pragma unroll
            for (int j = 0; j < V; ++j) p[j] = c * pr[j];
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) p[j] = val * pr[j];
        }
        // segmented inclusive scan over the SW slots (segments = equal rows)
        const int prow = __shfl_up(row, LANES);
        const bool head = (slot == 0) || (prow != row);
        const uint64_t hm = __ballot(head && sub == 0);
        const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
        const int sstart = (63 - __clzll(hm & upto)) / LANES;
#pragma unroll
        for (int d = 1; d < SW; d <<= 1) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const float t = __shfl_up(p[j], d * LANES);
                if (slot - d >= sstart) p[j] += t;
            }
        }
        const int nrow = __shfl_down(row, LANES);
        const bool tail = (slot == SW - 1) || (nrow != row);
        const int row0 = __shfl(row, 0);
        if (row0 == carry_row) {
            if (sstart == 0) {
#pragma unroll
                for (int j = 0; j < V; ++j) p[j] += carry[j];
            }
        } else if (carry_row >= 0) {
            if (slot == 0 && ract) flush_mid(carry_row, carry);
        }
        if (tail && slot != SW - 1 && ract) flush_mid(row, p);
#pragma unroll
        for (int j = 0; j < V; ++j) carry[j] = __shfl(p[j], (SW - 1) * LANES + sub);
        carry_row = __shfl(row, (SW - 1) * LANES);
    }
    // the shard's last row: complete, or a partial (first or last slot)
    if (slot == 0 && ract) {
        const bool split_after = a.row_ptr[l + 1] > end;
        float *dst;
        if (l == f && split_before) dst = cbase;
        else if (split_after) dst = cbase + (l == f ? 0 : R);
        else dst = a.out + (int64_t)l * R;
        store_row<V, STRIDED>(dst, R, sub, carry);
    }
}

// ---- sampled CP loss forward: one double partial per shard ---------------
template <int N, typename FT, int LANES, int V, bool STRIDED>
__global__ __launch_bounds__(256) void loss_kernel(Args a)
{
    constexpr int SW = WAVE / LANES;
    const int lane = threadIdx.x & 63;
    const int sidx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sidx >= a.nshards) return;
    const int start = a.shards[3 * sidx];
    const int end = start + a.shards[3 * sidx + 1];
    const int R = a.R;
    const int slot = lane / LANES, sub = lane % LANES;
    const bool ract = lane_active<LANES, V, STRIDED>(sub, R);
    double acc = 0.0;
    for (int base = start; base < end; base += SW) {
        const int e = base + slot;
        float m = 0.0f, val = 0.0f;
        if (e < end) {
            const Rec<N> rc = load_rec<N>(a.rin, e);
            val = __uint_as_float(rc.w[N]);
            if (ract) {
                float pr[V];
                row_product<N, FT, V, STRIDED>(a, rc, -1, sub, pr);
#pragma unroll
                for (int j = 0; j < V; ++j) m += pr[j];
            }
        }
        m = slot_sum<LANES>(m);
        if (e < end && sub == 0) {
            const float rho = val - m;
            acc += (double)(rho * rho);    // FP32 term, FP64 accumulation
        }
    }
    acc = wave_sum_d(acc);
    if (lane == 0) a.partial[sidx] = acc;
}

// ---- standalone remap: L_{n+1}[P_n[i]] = L_n[i] -------------------------
template <int N>
__global__ void remap_kernel(const uint32_t *__restrict__ rin, uint32_t *__restrict__ rout,
                             const int32_t *__restrict__ perm, int64_t nnz)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x)
        store_rec<N>(rout, perm[i], load_rec<N>(rin, i));
}

}  // namespace mk
