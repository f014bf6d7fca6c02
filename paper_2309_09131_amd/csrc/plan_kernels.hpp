// Integer preprocessing kernels (plan): index validation, stable LSD radix
// sort of positions by one coordinate, permutation inversion, row pointers,
// packing of the mode-0 layout.  No global atomics: per-tile histograms,
// a device-wide exclusive scan, and an order-preserving per-tile scatter.
#pragma once
#include "common.hpp"

namespace plan {

constexpr int TILE = 4096;          // items per radix tile
constexpr int SCAN_CHUNK = 1024;    // items per scan block (256 threads x 4)

// err[0] = 1 if any coordinate of mode n is outside [0, dims[n]).
struct Dims8 { int32_t d[8]; };

__global__ void validate_kernel(const int32_t *__restrict__ idx, int nmodes, int64_t nnz,
                                Dims8 dims, int32_t *__restrict__ err)
{
    int64_t total = nnz * nmodes;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int n = (int)(t / nnz);
        int32_t c = idx[t];
        if (c < 0 || c >= dims.d[n]) err[0] = 1;   // benign same-value race
    }
}

// keys[j] = coord[src[j]] (src == nullptr: identity); vals[j] = j when
// iota is set, else src[j].
__global__ void gather_keys_kernel(const int32_t *__restrict__ coord,
                                   const int32_t *__restrict__ src, int64_t n,
                                   int32_t *__restrict__ keys, int32_t *__restrict__ vals,
                                   int iota)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = src ? src[j] : (int32_t)j;
        keys[j] = coord[s];
        vals[j] = iota ? (int32_t)j : s;
    }
}

// Per-tile digit histogram, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(256) void radix_upsweep(const int32_t *__restrict__ keys,
                                                     int64_t n, int shift,
                                                     int32_t *__restrict__ hist, int ntiles)
{
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * TILE;
    for (int k = threadIdx.x; k < TILE; k += 256) {
        int64_t j = base + k;
        if (j < n) atomicAdd(&cnt[(keys[j] >> shift) & 255], 1);   // LDS atomic
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan, three phases over chunks of SCAN_CHUNK.
__device__ __forceinline__ int32_t block_excl_scan256(int32_t v, int32_t *sh, int32_t *total)
{
    // inclusive scan within waves, then across the 4 waves
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t t = __shfl_up(x, d);
        if (lane >= d) x += t;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int32_t off = 0;
    for (int k = 0; k < w; ++k) off += sh[k];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(256) void scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                   int32_t *__restrict__ sums)
{
    __shared__ int32_t sh[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int32_t v = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t j = base + threadIdx.x * 4 + k;
        if (j < n) v += in[j];
    }
    int32_t tot;
    block_excl_scan256(v, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of `n` chunk sums in place (sequential over
// groups of 1024).
__global__ __launch_bounds__(256) void scan_sums(int32_t *__restrict__ sums, int64_t n)
{
    __shared__ int32_t sh[4];
    int32_t carry = 0;
    for (int64_t base = 0; base < n; base += SCAN_CHUNK) {
        int32_t v[4], s = 0;
        for (int k = 0; k < 4; ++k) {
            int64_t j = base + threadIdx.x * 4 + k;
            v[k] = (j < n) ? sums[j] : 0;
            s += v[k];
        }
        int32_t tot;
        int32_t ex = block_excl_scan256(s, sh, &tot);
        int32_t run = carry + ex;
        for (int k = 0; k < 4; ++k) {
            int64_t j = base + threadIdx.x * 4 + k;
            if (j < n) sums[j] = run;
            run += v[k];
        }
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                  const int32_t *__restrict__ sums,
                                                  int32_t *__restrict__ out)
{
    __shared__ int32_t sh[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t j = base + threadIdx.x * 4 + k;
        v[k] = (j < n) ? in[j] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t run = sums[blockIdx.x] + block_excl_scan256(s, sh, &tot);
    for (int k = 0; k < 4; ++k) {
        int64_t j = base + threadIdx.x * 4 + k;
        if (j < n) out[j] = run;
        run += v[k];
    }
}

// Stable scatter of one tile by four waves, with coalesced writes.  Wave w
// ranks the items [w*1024, (w+1)*1024) of the tile in 16 rounds of 64 with
// ballot matching (equal digits keep their order) and counts its digits;
// the tile's items are then placed in LDS in (digit, position) order and
// written out so that consecutive threads write consecutive addresses of a
// digit's run.
__global__ __launch_bounds__(256) void radix_scatter_tile(const int32_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin,
                                                          int64_t n, int shift,
                                                          const int32_t *__restrict__ offs,
                                                          int ntiles, int32_t *__restrict__ kout,
                                                          int32_t *__restrict__ vout)
{
    constexpr int PER = TILE / 256;           // rounds per wave (16)
    __shared__ int32_t skey[TILE], sval[TILE];
    __shared__ int32_t wcnt[4][256];          // digit counts per wave, then prefixes
    __shared__ int32_t tpre[256];             // tile-local start of each digit
    __shared__ int32_t gbase[256];            // global start of each digit (this tile)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int d = t; d < 256; d += 256) {
        gbase[d] = offs[(int64_t)d * ntiles + blockIdx.x];
        wcnt[0][d] = wcnt[1][d] = wcnt[2][d] = wcnt[3][d] = 0;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t t0 = (int64_t)blockIdx.x * TILE + (int64_t)w * (TILE / 4);
    int32_t k[PER], v[PER], dg[PER], rk[PER];
    bool ok[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int64_t j = t0 + q * 64 + lane;
        ok[q] = j < n;
        k[q] = ok[q] ? kin[j] : 0;
        v[q] = ok[q] ? vin[j] : 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int d = (k[q] >> shift) & 255;
        uint64_t peers = __ballot(ok[q]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bits = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bits : ~bits;
        }
        dg[q] = d;
        rk[q] = ok[q] ? wcnt[w][d] + __popcll(peers & lt) : 0;
        // the highest lane of each digit group advances the wave's count
        // (only this wave touches wcnt[w]; lanes of one round write
        // different digits)
        const bool leader = ok[q] && ((peers >> lane) == 1ull);
        __builtin_amdgcn_wave_barrier();
        if (leader) wcnt[w][d] += __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // prefixes: per digit over the waves, and over the digits of the tile
    {
        const int d = t;                      // 256 threads, one digit each
        int c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
        const int tot = c0 + c1 + c2 + c3;
        int x = tot;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int y = __shfl_up(x, dd);
            if (lane >= dd) x += y;
        }
        __shared__ int32_t wsum[4];
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int off = 0;
        for (int q = 0; q < w; ++q) off += wsum[q];
        tpre[d] = off + x - tot;
        wcnt[0][d] = 0;
        wcnt[1][d] = c0;
        wcnt[2][d] = c0 + c1;
        wcnt[3][d] = c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (ok[q]) {
            const int pos = tpre[dg[q]] + wcnt[w][dg[q]] + rk[q];
            skey[pos] = k[q];
            sval[pos] = v[q];
        }
    __syncthreads();
    const int64_t left = n - (int64_t)blockIdx.x * TILE;
    const int cnt = left < TILE ? (int)left : TILE;
    for (int p = t; p < cnt; p += 256) {
        const int32_t key = skey[p];
        const int d = (key >> shift) & 255;
        const int64_t g = (int64_t)gbase[d] + (p - tpre[d]);
        kout[g] = key;
        vout[g] = sval[p];
    }
}

// P[q[t]] = t ; onew[t] = oold[q[t]]   (q = positions of L_n in L_{n+1} order)
__global__ void invert_kernel(const int32_t *__restrict__ q, int64_t n, int32_t *__restrict__ P,
                              const int32_t *__restrict__ oold, int32_t *__restrict__ onew)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = q[t];
        P[s] = (int32_t)t;
        onew[t] = oold[s];
    }
}

// Locality order (plan option): a 31-bit slice, from bit `shift`, of the
// Morton code of two coordinates (bit k of a at bit 2k+1, of b at bit 2k)
// of input src[j] (or j), as a radix-sort key; vals[j] = that input.
__device__ __forceinline__ uint64_t spread_even(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

__global__ void morton_keys_kernel(const int32_t *__restrict__ ca, const int32_t *__restrict__ cb,
                                   const int32_t *__restrict__ src, int64_t n, int shift,
                                   int32_t *__restrict__ keys, int32_t *__restrict__ vals)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = src ? src[j] : (int32_t)j;
        const uint64_t z = (spread_even((uint32_t)ca[s]) << 1) | spread_even((uint32_t)cb[s]);
        keys[j] = (int32_t)((z >> shift) & 0x7fffffffull);
        vals[j] = s;
    }
}

// slot[ord[j]] = j: the position of each input in a layout.
__global__ void slot_of_kernel(const int32_t *__restrict__ ord, int64_t n,
                               int32_t *__restrict__ slot)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        slot[ord[j]] = (int32_t)j;
}

// P[i] = slot[ord[i]]: the slot, in the next layout, of slot i's element.
__global__ void compose_kernel(const int32_t *__restrict__ slot, const int32_t *__restrict__ ord,
                               int64_t n, int32_t *__restrict__ P)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        P[i] = slot[ord[i]];
}

// Row pointers of a layout sorted by the mode's coordinate: row_ptr[r] =
// first position whose coordinate is >= r (= number of nonzeros with
// coordinate < r), r = 0..I, by a binary search of the coordinates in
// layout order.  One thread per row, every entry written once, so a long
// run of empty rows costs no more than any other rows.
__global__ void row_ptr_kernel(const int32_t *__restrict__ sorted, int64_t n, int32_t I,
                               int32_t *__restrict__ row_ptr)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= I;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;                 // first position with sorted[pos] >= r
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted[mid] < r) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[r] = (int32_t)lo;
    }
}

}  // namespace plan
