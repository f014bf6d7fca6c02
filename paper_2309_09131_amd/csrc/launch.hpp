// Kernel argument block and the per-mode-count launchers.  Each launcher is
// defined (explicitly specialised) in inst_n<N>.hip, one translation unit
// per number of modes, so the template kernels compile in parallel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mk {

// Row-start table of a layout L_m (built by the plan): for each block of 64
// consecutive positions, three words {bits 0-31, bits 32-63, count}: bit j
// is set when position 64b + j is the first of an output row, and count is
// the number of rows that start before the block.  With the list of the
// mode's nonempty rows in order, the output row of position e is
// rows[count + popcount(bits up to and including j) - 1].  The records of
// L_m omit c_m, which this recovers.
constexpr int RS_WORDS = 3;

struct Args {
    const uint32_t *rin;      // L_n records
    uint32_t *rout;           // L_{n+1} records, or nullptr (no remap)
    const int32_t *perm;      // P_n
    const int32_t *row_ptr;   // I_n + 1
    const int32_t *shards;    // [nshards][3] = start, len, super-shard
    const int32_t *fl;        // [nshards][2] = first and last output row
    const int32_t *order;     // dispatch order of shards, or nullptr
    const uint32_t *rbits;    // row-start table of L_n
    const int32_t *nrows;     // nonempty rows of mode n, ascending
    int32_t nblk;             // last valid index of the row-start table
    int32_t nshards;
    int32_t mode;
    int32_t R;
    int32_t cw;               // coordinate words per record (W)
    const void *fac[8];       // factor matrices (I_w x R row-major)
    float *out;               // I_n x R
    float *carry;             // [nshards][2][R] boundary partials
    const double *gscale;     // residual variant: upstream scale or nullptr
    double *partial;          // loss forward: one double per shard
    uint32_t coff[8];         // bit offset of each coordinate in an L_n record
    uint32_t ooff[8];         // ... in an L_{n+1} record (in-kernel remap)
    uint32_t cmask[8];        // its mask, 2^b - 1
};

// The standalone remap L_n -> L_{n+1}: c_n re-inserted from L_n's row-start
// table, c_{n+1} dropped.
struct RemapMap {
    uint32_t ioff[8];         // bit offsets in an L_n record
    uint32_t ooff[8];         // bit offsets in an L_{n+1} record
    uint32_t msk[8];
    const uint32_t *rbits;    // row-start table of L_n
    const int32_t *nrows;     // nonempty rows of mode n
    // per region of 64 * remap_rt_of(W, small) positions of L_n (one wave's
    // records): the ids of the rows its positions lie in, from the row
    // holding its first position on (64 entries; -1 in the first when the
    // region covers more than 64 rows)
    const int32_t *rids;
    int32_t nblk;
    int32_t n, nx;
    int32_t small;            // records per thread: remap_rt_of(W, small)
    // the same move as one bit-string operation on records of at most three
    // coordinate words (x their coordinate bits, as a 64- or 128-bit
    // integer): y = (x & (2^ba - 1)) | (hi ? (x >> bh) << bu : 0)
    // | (c_n << bp).  The fields below c_nx's stay, c_nx's is dropped, the
    // fields above it move to make room for c_n; every shift is below the
    // integer's width (hi = 0 when no field lies above c_nx's).
    uint32_t ba, bh, bu, bp, hi;
};

// Records per thread of the standalone remap for W coordinate words.  The
// large form: 32 for 8-byte records, 24 for 12-byte ones, else 16, fewer
// when the LDS stage of 256 * RT records plus their targets would exceed
// 96 KB (one block per CU); it combines the most partly written lines, for
// remaps into modes with many rows.  The small form: at most 16, and a
// stage within 72 KB (76 KB with the bucket counters), so that two blocks
// share a CU and one block's
// arithmetic overlaps the other's loads, for remaps into modes with few
// rows, which run near the copy rate.
__host__ __device__ constexpr int remap_rt_of(int W, bool small)
{
    // large: 16 measured fastest of 8, 12, 16, 24 and 30 for 16-byte
    // records, 24 for 12-byte ones, 32 for 8-byte ones (16% faster than 16)
    return small ? ((72 * 1024) / (256 * (4 * (W + 1) + 4)) < 16
                        ? (72 * 1024) / (256 * (4 * (W + 1) + 4))
                        : 16)
                 : (((W + 1 == 2) ? 32 : (W + 1 == 3) ? 24 : 16) <
                            (96 * 1024) / (256 * (4 * (W + 1) + 4))
                        ? ((W + 1 == 2) ? 32 : (W + 1 == 3) ? 24 : 16)
                        : (96 * 1024) / (256 * (4 * (W + 1) + 4)));
}

// Remaps into a mode with at most this many rows use the small form
// (measured on the 4-mode workload: into 2K rows 0.87 -> 0.61 ms, into 20K
// 0.93 -> 0.87 ms; into 500K and 1M rows the large form is 5% faster).
constexpr int64_t REMAP_SMALL_ROWS = int64_t(1) << 16;

// Record widths compiled for N modes: W coordinate words with
// rec_wmin(N) <= W <= N - 1 (the host rounds the packed width up into this
// range).  A record holds the N - 1 coordinates other than its layout's
// output mode, so W = N - 1 holds any coordinates; the narrower forms cover
// the common case of coordinates well below 2^31.
__host__ __device__ constexpr int rec_wmin(int N)
{
    return N >= 5 ? N - 3 : (N == 4 ? 2 : 1);
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
                        int cw, const RemapMap &rm, hipStream_t s);
// Bit offsets of the coordinates in an L_0 record; mode `skip` (0, the
// layout's output mode) is not stored.
struct PackMap {
    uint32_t off[8];
    int32_t skip;
};
template <int N>
hipError_t launch_pack(const int32_t *idx, const float *vals, const int32_t *o, int64_t nnz,
                       uint32_t *rec, int cw, PackMap pm, hipStream_t s);

#define MK_DECLARE(N)                                                                      \
    template <>                                                                            \
    hipError_t launch_mttkrp<N>(const Args &, int, LaneCfg, int, unsigned, hipStream_t);   \
    template <>                                                                            \
    hipError_t launch_remap<N>(const uint32_t *, uint32_t *, const int32_t *, int64_t,     \
                               int, const RemapMap &, hipStream_t);                        \
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
