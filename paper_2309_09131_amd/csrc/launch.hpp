// Kernel argument block and the per-mode-count launchers.  Each launcher is
// defined (explicitly specialised) in inst_n<N>.hip, one translation unit
// per number of modes, so the template kernels compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mk {

struct Args {
    const uint32_t *rin;      // L_n records
    uint32_t *rout;           // L_{n+1} records, or nullptr (no remap)
    const int32_t *perm;      // P_n
    const int32_t *row_ptr;   // I_n + 1
    const int32_t *shards;    // [nshards][3] = start, len, super-shard
    const int32_t *order;     // dispatch order of shards, or nullptr
    int32_t nshards;
    int32_t mode;
    int32_t R;
    int32_t cw;               // coordinate words per record (W)
    const void *fac[8];       // factor matrices (I_w x R row-major)
    float *out;               // I_n x R
    float *carry;             // [nshards][2][R] boundary partials
    const double *gscale;     // residual variant: upstream scale or nullptr
    double *partial;          // loss forward: one double per shard
    uint32_t coff[8];         // bit offset of each mode's coordinate in a record
    uint32_t cmask[8];        // its mask, 2^b - 1
};

// Record widths compiled for N modes: W coordinate words with
// rec_wmin(N) <= W <= N (the host rounds the packed width up into this
// range).  W = N holds any coordinates; the narrower forms cover the
// common case of coordinates well below 2^31.
__host__ __device__ constexpr int rec_wmin(int N)
{
    return N >= 5 ? N - 2 : (N >= 2 ? N - 1 : 1);
}

// Waves (one shard each) per workgroup of the MTTKRP kernels (1, 2 and 4
// measured equal; 8 and 12 slower).
constexpr int MTT_WAVES = 4;

// Lane configuration: contiguous (lanes = nextpow2(R / V); j = 2: V = 32
// bytes of factor row per lane, j = 1: 16 bytes) or strided (64 lanes,
// j = ceil(R / 64) ranks each).
struct LaneCfg {
    int lanes;
    int j;
    bool strided;
};

// KIND_GATHER: the MTTKRP kernel's loads without its segmented reduction
// (measurement only; contiguous lane forms).  KIND_RESID_LOSS: the residual
// pass that also sums the squared residuals (loss and gradient in one pass).
enum Kind { KIND_MTTKRP = 0, KIND_RESID = 1, KIND_LOSS = 2, KIND_GATHER = 3,
            KIND_RESID_LOSS = 4 };

template <int N>
hipError_t launch_mttkrp(const Args &a, int bf16, LaneCfg c, int kind, unsigned grid,
                         hipStream_t s);
template <int N>
hipError_t launch_remap(const uint32_t *rin, uint32_t *rout, const int32_t *perm, int64_t nnz,
                        int cw, hipStream_t s);
// Bit offsets of the coordinates in a packed record.
struct PackMap {
    uint32_t off[8];
};
template <int N>
hipError_t launch_pack(const int32_t *idx, const float *vals, const int32_t *o, int64_t nnz,
                       uint32_t *rec, int cw, PackMap pm, hipStream_t s);

#define MK_DECLARE(N)                                                                      \
    template <>                                                                            \
    hipError_t launch_mttkrp<N>(const Args &, int, LaneCfg, int, unsigned, hipStream_t);   \
    template <>                                                                            \
    hipError_t launch_remap<N>(const uint32_t *, uint32_t *, const int32_t *, int64_t,     \
                               int, hipStream_t);                                          \
    template <>                                                                            \
    hipError_t launch_pack<N>(const int32_t *, const float *, const int32_t *, int64_t,    \
                              uint32_t *, int, PackMap, hipStream_t);
MK_DECLARE(2)
MK_DECLARE(3)
MK_DECLARE(4)
MK_DECLARE(5)
MK_DECLARE(6)
MK_DECLARE(7)
MK_DECLARE(8)
#undef MK_DECLARE

}  // namespace mk
