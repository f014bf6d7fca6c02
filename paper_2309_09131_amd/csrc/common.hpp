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

// The same coordinate read straight from record i of a buffer.
template <int W>
__device__ __forceinline__ int rec_coord_at(const uint32_t *__restrict__ buf, int64_t i,
                                            uint32_t off, uint32_t mask)
{
    const uint32_t *p = buf + i * (W + 1) + (off >> 5);
    const uint64_t x = ((uint64_t)p[1] << 32) | p[0];
    return (int)((uint32_t)(x >> (off & 31u)) & mask);
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
