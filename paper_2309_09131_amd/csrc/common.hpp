// Shared device helpers for the gfx950 kernels: packed nonzero records,
// BF16 <-> FP32 conversion, wave64 shuffles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define WAVE 64

// One nonzero: W words holding the N coordinates bit-packed, followed by
// the FP32 value (4W + 4 bytes).  Coordinate n occupies bits [off_n,
// off_n + b_n) of the W words read as one little-endian bit string, b_n
// being the bit length of I_n - 1; a coordinate may straddle two words.
// Records are 4-byte aligned; gfx950 global loads/stores of 8 or 16 bytes
// only need dword alignment, so the compiler emits wide accesses.
template <int W>
struct Rec {
    uint32_t w[W + 1];
};

template <int W>
__device__ __forceinline__ Rec<W> load_rec(const uint32_t *__restrict__ buf, int64_t i)
{
    // word by word: keeps the record in registers (a struct copy through a
    // reinterpreted pointer made the compiler stage record arrays in LDS);
    // adjacent dwords are still merged into wide loads
    Rec<W> r;
    const uint32_t *p = buf + i * (W + 1);
#pragma unroll
    for (int k = 0; k < W + 1; ++k) r.w[k] = p[k];
    return r;
}

template <int W>
__device__ __forceinline__ void store_rec(uint32_t *__restrict__ buf, int64_t i, const Rec<W> &r)
{
    *reinterpret_cast<Rec<W> *>(buf + i * (W + 1)) = r;
}

// Streaming variant (non-temporal hint, per dword) for a read-once record stream.
template <int W>
__device__ __forceinline__ Rec<W> load_rec_nt(const uint32_t *__restrict__ buf, int64_t i)
{
    Rec<W> r;
    const uint32_t *p = buf + i * (W + 1);
#pragma unroll
    for (int k = 0; k < W + 1; ++k) r.w[k] = __builtin_nontemporal_load(p + k);
    return r;
}

// The coordinate at bit offset `off` (runtime, uniform) with mask `mask`
// (2^b - 1) of a record held in registers, without dynamic register
// indexing, which would push the record to scratch memory: the two words
// that can hold it are picked with selects on the uniform word index (one
// select per word and half; and-or masks measured 2-3% slower in the MTTKRP
// kernel), then shifted as one 64-bit value.  The second word may be the
// value word, whose bits the mask removes.
template <int W>
__device__ __forceinline__ int rec_coord(const Rec<W> &r, uint32_t off, uint32_t mask)
{
    const uint32_t q = off >> 5;
    uint32_t lo = r.w[0], hi = r.w[1];
#pragma unroll
    for (int k = 1; k < W; ++k) {
        lo = (q == (uint32_t)k) ? r.w[k] : lo;
        hi = (q == (uint32_t)k) ? r.w[k + 1] : hi;
    }
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    return (int)((uint32_t)(x >> (off & 31u)) & mask);
}

// Or a coordinate (which fits its field) into the field at bit offset
// `off` of a record being built (its coordinate words zeroed first).
template <int W>
__device__ __forceinline__ void rec_put(Rec<W> &r, uint32_t off, uint32_t v)
{
    const uint32_t q = off >> 5;
    const uint64_t x = (uint64_t)v << (off & 31u);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        r.w[k] |= (q == (uint32_t)k) ? (uint32_t)x : 0u;
        r.w[k] |= (q + 1 == (uint32_t)k) ? (uint32_t)(x >> 32) : 0u;
    }
}

// An L_n record in L_{n+1}'s format: the coordinates of the modes other than
// n and nx move from their L_n fields (ioff) to their L_{n+1} fields (ooff),
// the output row c_n (implied by the position in L_n, passed in `row`) is
// stored, and c_nx (implied by the position in L_{n+1}) is dropped.
template <int N, int W>
__device__ __forceinline__ Rec<W> repack(const Rec<W> &r, int row, int n, int nx,
                                         const uint32_t *ioff, const uint32_t *ooff,
                                         const uint32_t *msk)
{
    Rec<W> o;
#pragma unroll
    for (int k = 0; k < W; ++k) o.w[k] = 0u;
    o.w[W] = r.w[W];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        if (m == nx) continue;
        const uint32_t v = (m == n) ? (uint32_t)row : (uint32_t)rec_coord<W>(r, ioff[m], msk[m]);
        rec_put<W>(o, ooff[m], v);
    }
    return o;
}

// Row-start table lookups (layout described in launch.hpp): the ordinal of
// the output row holding position e among the mode's nonempty rows, and
// whether e is the first position of that row, from the table entry
// {lo, hi, count} of e's block.
struct RowStart {
    uint32_t lo, hi, cnt;
};

__device__ __forceinline__ RowStart row_start_at(const uint32_t *__restrict__ t, int b)
{
    const uint32_t *q = t + 3 * (int64_t)b;
    return RowStart{q[0], q[1], q[2]};
}

__device__ __forceinline__ int row_ordinal(const RowStart &r, int e, bool &first)
{
    const int j = e & 63;
    const uint64_t bits = ((uint64_t)r.hi << 32) | r.lo;
    first = ((bits >> j) & 1ull) != 0;
    return (int)r.cnt + (int)__popcll(bits & ((2ull << j) - 1ull)) - 1;
}

// Row starts among the 64 positions from offset `off` (0..63) into table
// block b, from the entries of blocks b and b + 1: bit i of `m` is set when
// the position i places on starts a row; `before` counts the rows starting
// before the first of them.
struct SegStarts {
    uint64_t m;
    int before;
};

__device__ __forceinline__ SegStarts seg_starts(const RowStart &a, const RowStart &b, int off)
{
    const uint64_t ba = ((uint64_t)a.hi << 32) | a.lo, bb = ((uint64_t)b.hi << 32) | b.lo;
    SegStarts s;
    s.m = off ? ((ba >> off) | (bb << (64 - off))) : ba;
    s.before = (int)a.cnt + (int)__popcll(ba & ((1ull << off) - 1ull));
    return s;
}

// bfloat16 storage <-> float.  Widening is exact (the 16 high bits).
__device__ __forceinline__ float bf16lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __shfl_xor(lo, m);
    hi = __shfl_xor(hi, m);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
    return v;
}

static inline int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }
