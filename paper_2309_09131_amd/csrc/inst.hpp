// Instantiation of the templated kernels for one mode count NM (defined by
// the including inst_n<NM>.hip).
#pragma once
#include "mttkrp_kernels.hpp"

namespace plan {

// L_0 records: rec[j] = (coords of input o[j], value of input o[j]).
template <int N>
__global__ void pack_kernel(const int32_t *__restrict__ idx, const float *__restrict__ vals,
                            const int32_t *__restrict__ o, int64_t n, uint32_t *__restrict__ rec)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = o[j];
        Rec<N> r;
#pragma unroll
        for (int m = 0; m < N; ++m) r.w[m] = (uint32_t)idx[(int64_t)m * n + s];
        r.w[N] = __float_as_uint(vals[s]);
        store_rec<N>(rec, j, r);
    }
}

}  // namespace plan

namespace mk {

namespace {
template <typename FT, int LANES, int V, bool STRIDED>
hipError_t launch_one(const Args &a, int kind, unsigned grid, hipStream_t s)
{
    // separate instantiations with and without the in-kernel remap
    if (kind == KIND_MTTKRP && a.rout)
        hipLaunchKernelGGL((mttkrp_kernel<NM, FT, LANES, V, STRIDED, false, true>), dim3(grid),
                           dim3(MTT_WAVES * 64), 0, s, a);
    else if (kind == KIND_MTTKRP)
        hipLaunchKernelGGL((mttkrp_kernel<NM, FT, LANES, V, STRIDED, false, false>), dim3(grid),
                           dim3(MTT_WAVES * 64), 0, s, a);
    else if (kind == KIND_RESID && a.rout)
        hipLaunchKernelGGL((mttkrp_kernel<NM, FT, LANES, V, STRIDED, true, true>), dim3(grid),
                           dim3(MTT_WAVES * 64), 0, s, a);
    else if (kind == KIND_RESID)
        hipLaunchKernelGGL((mttkrp_kernel<NM, FT, LANES, V, STRIDED, true, false>), dim3(grid),
                           dim3(MTT_WAVES * 64), 0, s, a);
    else
        hipLaunchKernelGGL((loss_kernel<NM, FT, LANES, V, STRIDED>), dim3(grid), dim3(256), 0,
                           s, a);
    return hipGetLastError();
}

template <typename FT, int V>
hipError_t launch_contig(const Args &a, int lanes, int kind, unsigned grid, hipStream_t s)
{
    switch (lanes) {
    case 1: return launch_one<FT, 1, V, false>(a, kind, grid, s);
    case 2: return launch_one<FT, 2, V, false>(a, kind, grid, s);
    case 4: return launch_one<FT, 4, V, false>(a, kind, grid, s);
    case 8: return launch_one<FT, 8, V, false>(a, kind, grid, s);
    case 16: return launch_one<FT, 16, V, false>(a, kind, grid, s);
    case 32: return launch_one<FT, 32, V, false>(a, kind, grid, s);
    case 64:
        if constexpr (V == 4 && sizeof(FT) == 4) return launch_one<FT, 64, V, false>(a, kind, grid, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename FT>
hipError_t launch_strided(const Args &a, int j, int kind, unsigned grid, hipStream_t s)
{
    switch (j) {
    case 1: return launch_one<FT, 64, 1, true>(a, kind, grid, s);
    case 2: return launch_one<FT, 64, 2, true>(a, kind, grid, s);
    case 3: return launch_one<FT, 64, 3, true>(a, kind, grid, s);
    case 4: return launch_one<FT, 64, 4, true>(a, kind, grid, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

template <>
hipError_t launch_mttkrp<NM>(const Args &a, int bf16, LaneCfg c, int kind, unsigned grid,
                             hipStream_t s)
{
    if (c.strided)
        return bf16 ? launch_strided<uint16_t>(a, c.j, kind, grid, s)
                    : launch_strided<float>(a, c.j, kind, grid, s);
    // c.j selects the per-lane width for contiguous lanes: 1 = 16 bytes, 2 = 32
    if (bf16) {
        if (c.j == 2) return launch_contig<uint16_t, 16>(a, c.lanes, kind, grid, s);
        return launch_contig<uint16_t, 8>(a, c.lanes, kind, grid, s);
    }
    if (c.j == 2) return launch_contig<float, 8>(a, c.lanes, kind, grid, s);
    return launch_contig<float, 4>(a, c.lanes, kind, grid, s);
}

template <>
hipError_t launch_remap<NM>(const uint32_t *rin, uint32_t *rout, const int32_t *perm,
                            int64_t nnz, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    // one block per chunk of 256 * RT records (RT as in remap_kernel), the
    // grid rounded up to a multiple of the 8 XCDs
    constexpr int RT = remap_rt<NM>();
    const int64_t nchunks = (nnz + 256 * RT - 1) / (256 * RT);
    unsigned grid = (unsigned)(((nchunks + 7) / 8) * 8);
    hipLaunchKernelGGL((remap_kernel<NM>), dim3(grid), dim3(256), 0, s, rin, rout, perm, nnz);
    return hipGetLastError();
}

template <>
hipError_t launch_pack<NM>(const int32_t *idx, const float *vals, const int32_t *o,
                           int64_t nnz, uint32_t *rec, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    unsigned grid = (unsigned)((nnz + 255) / 256 < 65536 ? (nnz + 255) / 256 : 65536);
    hipLaunchKernelGGL((plan::pack_kernel<NM>), dim3(grid), dim3(256), 0, s, idx, vals, o, nnz,
                       rec);
    return hipGetLastError();
}

}  // namespace mk
