// Instantiation of the templated kernels for one mode count NM (defined by
// the including inst_n<NM>.hip), for every record width W of that mode
// count (rec_wmin(NM) <= W <= NM - 1 coordinate words).
#pragma once
#include "mttkrp_kernels.hpp"

namespace plan {

// L_0 records: rec[j] = (coordinates of input o[j] except c_0, which the
// position implies, bit-packed at the offsets pm.off, value of input o[j]).
// Every coordinate fits its field (the host sizes the fields from the
// dimensions and validates the input first), so the fields are simply or-ed
// in.
template <int N, int W>
__global__ void pack_kernel(const int32_t *__restrict__ idx, const float *__restrict__ vals,
                            const int32_t *__restrict__ o, int64_t n, mk::PackMap pm,
                            uint32_t *__restrict__ rec)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = o[j];
        Rec<W> r;
#pragma unroll
        for (int k = 0; k < W; ++k) r.w[k] = 0u;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            if (m == pm.skip) continue;
            const uint32_t q = pm.off[m] >> 5;
            const uint64_t x = (uint64_t)(uint32_t)idx[(int64_t)m * n + s] << (pm.off[m] & 31u);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                r.w[k] |= (q == (uint32_t)k) ? (uint32_t)x : 0u;
                r.w[k] |= (q + 1 == (uint32_t)k) ? (uint32_t)(x >> 32) : 0u;
            }
        }
        r.w[W] = __float_as_uint(vals[s]);
        store_rec<W>(rec, j, r);
    }
}

}  // namespace plan

namespace mk {

namespace {
template <int W, typename FT, int LANES, int V, bool STRIDED>
hipError_t launch_one(const Args &a, int kind, unsigned grid, hipStream_t s)
{
    // separate instantiations with and without the in-kernel remap
    const dim3 blk(MTT_WAVES * 64);
    if (kind == KIND_MTTKRP && a.rout)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_MTTKRP, true>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_MTTKRP)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_MTTKRP, false>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_RESID && a.rout)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_RESID, true>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_RESID)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_RESID, false>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_RESID_LOSS && !a.rout)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_RESID_LOSS, false>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_LOSS)
        hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_LOSS, false>),
                           dim3(grid), blk, 0, s, a);
    else if (kind == KIND_GATHER) {
        if constexpr (STRIDED) return hipErrorInvalidValue;
        else
            hipLaunchKernelGGL((mttkrp_kernel<NM, W, FT, LANES, V, STRIDED, KIND_GATHER, false>),
                               dim3(grid), blk, 0, s, a);
    } else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int W, typename FT, int V>
hipError_t launch_contig(const Args &a, int lanes, int kind, unsigned grid, hipStream_t s)
{
    switch (lanes) {
    case 1: return launch_one<W, FT, 1, V, false>(a, kind, grid, s);
    case 2: return launch_one<W, FT, 2, V, false>(a, kind, grid, s);
    case 4: return launch_one<W, FT, 4, V, false>(a, kind, grid, s);
    case 8: return launch_one<W, FT, 8, V, false>(a, kind, grid, s);
    case 16: return launch_one<W, FT, 16, V, false>(a, kind, grid, s);
    case 32: return launch_one<W, FT, 32, V, false>(a, kind, grid, s);
    case 64:
        if constexpr (V == 4 && sizeof(FT) == 4)
            return launch_one<W, FT, 64, V, false>(a, kind, grid, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <int W, typename FT>
hipError_t launch_strided(const Args &a, int j, int kind, unsigned grid, hipStream_t s)
{
    switch (j) {
    case 1: return launch_one<W, FT, 64, 1, true>(a, kind, grid, s);
    case 2: return launch_one<W, FT, 64, 2, true>(a, kind, grid, s);
    case 3: return launch_one<W, FT, 64, 3, true>(a, kind, grid, s);
    case 4: return launch_one<W, FT, 64, 4, true>(a, kind, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int W>
hipError_t launch_width(const Args &a, int bf16, LaneCfg c, int kind, unsigned grid,
                        hipStream_t s)
{
    if (c.strided)
        return bf16 ? launch_strided<W, uint16_t>(a, c.j, kind, grid, s)
                    : launch_strided<W, float>(a, c.j, kind, grid, s);
    // c.j selects the per-lane width for contiguous lanes: 1 = 16 bytes, 2 = 32
    if (bf16) {
        if (c.j == 2) return launch_contig<W, uint16_t, 16>(a, c.lanes, kind, grid, s);
        return launch_contig<W, uint16_t, 8>(a, c.lanes, kind, grid, s);
    }
    if (c.j == 2) return launch_contig<W, float, 8>(a, c.lanes, kind, grid, s);
    return launch_contig<W, float, 4>(a, c.lanes, kind, grid, s);
}

template <int W, int RT>
hipError_t launch_remap_rt(const uint32_t *rin, uint32_t *rout, const int32_t *perm,
                           int64_t nnz, const RemapMap &rm, hipStream_t s)
{
    // one block per chunk of 256 * RT records, the grid rounded up to a
    // multiple of the 8 XCDs
    const int64_t nchunks = (nnz + 256 * RT - 1) / (256 * RT);
    unsigned grid = (unsigned)(((nchunks + 7) / 8) * 8);
    hipLaunchKernelGGL((remap_kernel<NM, W, RT>), dim3(grid), dim3(256), 0, s, rin, rout, perm,
                       nnz, rm);
    return hipGetLastError();
}

template <int W>
hipError_t launch_remap_w(const uint32_t *rin, uint32_t *rout, const int32_t *perm, int64_t nnz,
                          const RemapMap &rm, hipStream_t s)
{
    if (rm.small) return launch_remap_rt<W, remap_rt_of(W, true)>(rin, rout, perm, nnz, rm, s);
    return launch_remap_rt<W, remap_rt_of(W, false)>(rin, rout, perm, nnz, rm, s);
}

template <int W>
hipError_t launch_pack_w(const int32_t *idx, const float *vals, const int32_t *o, int64_t nnz,
                         uint32_t *rec, PackMap pm, hipStream_t s)
{
    unsigned grid = (unsigned)((nnz + 255) / 256 < 65536 ? (nnz + 255) / 256 : 65536);
    hipLaunchKernelGGL((plan::pack_kernel<NM, W>), dim3(grid), dim3(256), 0, s, idx, vals, o,
                       nnz, pm, rec);
    return hipGetLastError();
}

// The compiled widths of this mode count: NM - 1, NM - 2 and NM - 3, never
// below rec_wmin(NM).
constexpr int W0 = NM - 1;
constexpr int W1 = NM - 2 >= rec_wmin(NM) ? NM - 2 : W0;
constexpr int W2 = NM - 3 >= rec_wmin(NM) ? NM - 3 : W1;
static_assert(rec_wmin(NM) >= NM - 3 && rec_wmin(NM) >= 1, "widths W0..W2 cover rec_wmin..NM-1");
}  // namespace

template <>
hipError_t launch_mttkrp<NM>(const Args &a, int bf16, LaneCfg c, int kind, unsigned grid,
                             hipStream_t s)
{
    if (a.cw == W0) return launch_width<W0>(a, bf16, c, kind, grid, s);
    if (a.cw == W1) return launch_width<W1>(a, bf16, c, kind, grid, s);
    if (a.cw == W2) return launch_width<W2>(a, bf16, c, kind, grid, s);
    return hipErrorInvalidValue;
}

template <>
hipError_t launch_remap<NM>(const uint32_t *rin, uint32_t *rout, const int32_t *perm,
                            int64_t nnz, int cw, const RemapMap &rm, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    if (cw == W0) return launch_remap_w<W0>(rin, rout, perm, nnz, rm, s);
    if (cw == W1) return launch_remap_w<W1>(rin, rout, perm, nnz, rm, s);
    if (cw == W2) return launch_remap_w<W2>(rin, rout, perm, nnz, rm, s);
    return hipErrorInvalidValue;
}

template <>
hipError_t launch_pack<NM>(const int32_t *idx, const float *vals, const int32_t *o,
                           int64_t nnz, uint32_t *rec, int cw, PackMap pm, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    if (cw == W0) return launch_pack_w<W0>(idx, vals, o, nnz, rec, pm, s);
    if (cw == W1) return launch_pack_w<W1>(idx, vals, o, nnz, rec, pm, s);
    if (cw == W2) return launch_pack_w<W2>(idx, vals, o, nnz, rec, pm, s);
    return hipErrorInvalidValue;
}

}  // namespace mk
