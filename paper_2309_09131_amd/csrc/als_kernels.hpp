// CP-ALS mode update in FP64 (Alg. "cp-als" with the standard normal-
// equation solve): Gram matrices G_w = A_w^T A_w, V = hadamard_{w != n} G_w,
// Cholesky V = L L^T, W = V^{-1} = L^{-T} L^{-1}, A_n = M_n W, column norms
// lambda, normalisation and storage (FP32 or BF16 round-to-nearest-even),
// fit reductions; plus the final sum of the sampled-loss partials.
// All reductions use a fixed partition and fixed order (deterministic).
#pragma once
#include "common.hpp"

namespace als {

constexpr int APPLY_BLOCKS = 2048;  // blocks (and partial rows) of apply kernels
constexpr int GRAM_TILE = 16;

template <typename FT>
__device__ __forceinline__ double ld(const FT *A, int64_t i);
template <>
__device__ __forceinline__ double ld<float>(const float *A, int64_t i) { return (double)A[i]; }
template <>
__device__ __forceinline__ double ld<uint16_t>(const uint16_t *A, int64_t i)
{
    return (double)bf16_to_f32(A[i]);
}

// Partial Gram over a row range: grid = (gb, tiles, tiles), 256 threads;
// block (b, y, z) computes the 16 x 16 tile p0 = 16 y, q0 = 16 z of
// part[b][p][q] = sum_{i in chunk b} A[i][p] A[i][q].
// The tile is a dense contraction over rows, so it runs on the FP64 matrix
// cores: one v_mfma_f64_16x16x4f64 adds X Y with X[p][k] = A[i_k][p0 + p]
// and Y[k][q] = A[i_k][q0 + q] for four rows i_k, and lane l supplies row
// i_{l/16} at column l % 16 of both operands (one coalesced 64-byte piece of
// each of the four rows).  Wave w of the block takes the rows
// i0 + 16 j + 4 w + k, eight steps of four rows in flight; the four waves'
// tiles are added in LDS in wave order.  Lane l then holds the tile entries
// (l / 16 + 4 v, l % 16), v = 0..3 (checked on the device against a CPU
// product).  Columns beyond R and rows beyond the chunk enter as zeros.
static_assert(GRAM_TILE == 16, "the Gram tile is one 16 x 16 FP64 MFMA tile");
template <typename FT>
__global__ __launch_bounds__(256) void gram_partial(const FT *__restrict__ A, int64_t I, int R,
                                                    int64_t chunk, double *__restrict__ part)
{
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double red[4][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = blockIdx.y * 16, q0 = blockIdx.z * 16;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < I) ? i0 + chunk : I;
    const int c = lane % 16, kr = lane / 16;
    const bool okp = p0 + c < R, okq = q0 + c < R;
    const int pc = okp ? p0 + c : R - 1, qc = okq ? q0 + c : R - 1;
    const bool diag = p0 == q0;                  // uniform: Y's values are X's
    constexpr int UN = 8;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t ib = i0 + 4 * w; ib < i1; ib += 16 * UN) {   // uniform trip count
        double a[UN], b[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t i = ib + 16 * u + kr;
            const bool ok = i < i1;
            const int64_t ic = ok ? i : i0;      // clamped: in bounds
            const double x = ld<FT>(A, ic * R + pc);
            a[u] = (ok && okp) ? x : 0.0;
            if (!diag) {
                const double y = ld<FT>(A, ic * R + qc);
                b[u] = (ok && okq) ? y : 0.0;
            } else {
                b[u] = a[u];
            }
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][(lane / 16 + 4 * v) * 16 + lane % 16] = acc[v];
    __syncthreads();
    const int t = threadIdx.x, ty = t / 16, tx = t % 16;
    if (p0 + ty < R && q0 + tx < R)
        part[((int64_t)blockIdx.x * R + p0 + ty) * R + q0 + tx] =
            ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// G[t] = sum_b part[b][t]: one block per entry, strided partial sums then a
// fixed tree (deterministic).
__global__ __launch_bounds__(64) void gram_reduce(const double *__restrict__ part, int gb, int R,
                                                 double *__restrict__ G)
{
    const int t = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < gb; b += 64) v += part[(int64_t)b * R * R + t];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
    if (threadIdx.x == 0) G[t] = v;
}

// One block of 256 threads.  V = hadamard_{w != n} G_w; Cholesky (lower) in
// place in L; if a pivot is not positive, restart once with the ridge
// 1e-12 * trace(V) / R on the diagonal (ridge counter += 1); then
// Linv = L^{-1} and W = Linv^T Linv.  fail[0] = 1 if even the ridge fails.
__global__ __launch_bounds__(256) void chol_inverse(const double *__restrict__ G, int nmodes,
                                                    int skip, int R, double *__restrict__ L,
                                                    double *__restrict__ Linv,
                                                    double *__restrict__ W,
                                                    int32_t *__restrict__ ridge,
                                                    int32_t *__restrict__ fail)
{
    __shared__ int bad;
    __shared__ double tr;
    const int t = threadIdx.x;
    for (int attempt = 0; attempt < 2; ++attempt) {
        for (int e = t; e < R * R; e += 256) {
            double v = 1.0;
            for (int w = 0; w < nmodes; ++w)
                if (w != skip) v *= G[(int64_t)w * R * R + e];
            L[e] = v;
        }
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int i = 0; i < R; ++i) s += L[i * R + i];
            tr = s;
            bad = 0;
        }
        __syncthreads();
        if (attempt == 1) {
            for (int i = t; i < R; i += 256) L[i * R + i] += 1e-12 * tr / R;
            __syncthreads();
        }
        for (int j = 0; j < R; ++j) {
            if (t == 0) {
                double d = L[j * R + j];
                if (!(d > 0.0)) bad = 1;
                L[j * R + j] = (d > 0.0) ? sqrt(d) : 1.0;
            }
            __syncthreads();
            const double djj = L[j * R + j];
            for (int i = j + 1 + t; i < R; i += 256) L[i * R + j] /= djj;
            __syncthreads();
            // trailing update of the lower triangle
            const int m = R - j - 1;
            for (int e = t; e < m * m; e += 256) {
                const int i = j + 1 + e / m, k = j + 1 + e % m;
                if (k <= i) L[i * R + k] -= L[i * R + j] * L[k * R + j];
            }
            __syncthreads();
        }
        if (!bad) break;
        if (attempt == 0 && t == 0) ridge[0] += 1;
        __syncthreads();
        if (attempt == 1 && t == 0) fail[0] = 1;
    }
    // upper triangle of L is zero
    for (int e = t; e < R * R; e += 256)
        if (e % R > e / R) L[e] = 0.0;
    __syncthreads();
    // column c of L^{-1} by forward substitution (one thread per column)
    for (int c = t; c < R; c += 256) {
        for (int i = 0; i < c; ++i) Linv[i * R + c] = 0.0;
        for (int i = c; i < R; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i * R + k] * Linv[k * R + c];
            Linv[i * R + c] = s / L[i * R + i];
        }
    }
    __syncthreads();
    for (int e = t; e < R * R; e += 256) {
        const int p = e / R, q = e % R;
        const int k0 = p > q ? p : q;
        double s = 0.0;
        for (int k = k0; k < R; ++k) s += Linv[k * R + p] * Linv[k * R + q];
        W[e] = s;
    }
}

// Round-to-odd FP64 -> FP32 keeps one later RNE rounding to BF16 correct.
__device__ __forceinline__ float to_f32_odd(double x)
{
    float f = __double2float_rz(x);
    if ((double)f != x) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f;
}

template <typename FT>
__device__ __forceinline__ void st(FT *A, int64_t i, double x);
template <>
__device__ __forceinline__ void st<float>(float *A, int64_t i, double x) { A[i] = (float)x; }
template <>
__device__ __forceinline__ void st<uint16_t>(uint16_t *A, int64_t i, double x)
{
    A[i] = f32_to_bf16_rne(to_f32_odd(x));
}

// X = M W row by row (FP64).  pass 0: colsq[block][r] = sum of X(i,r)^2 over
// the block's rows.  pass 1: A(i,r) = X(i,r) / lambda_r (lambda_r = 0: X).
// Threads: RT per row (RT >= R, a power of two), RP = 256 / RT rows at a
// time; thread (g, r) takes the rows i0 + g, i0 + g + RP, ... of its block
// in that order and sums X(i,r) over q = 0..R-1 in order, so the results do
// not depend on the form below.
//   R <= 32 (W in 8 KB of LDS): the RT lanes of a row, inside one wave, each
//   load one element of it, and X(i,r) takes M(i,q) from lane q by a
//   cross-lane read; each thread keeps four rows' loads in flight and the
//   loop has no barrier.  (Staging every RP rows in LDS between two barriers
//   left the kernel latency-bound at about 0.4 TB/s on a 2M-row factor.)
//   The small LDS footprint lets several blocks share a CU with the remap
//   kernel (96 KB of LDS) that runs beside this update.
//   R > 32: the RP rows are staged in LDS with one coalesced load each and W
//   is read from memory.
template <typename FT>
__global__ __launch_bounds__(256) void als_apply(const float *__restrict__ M, int64_t I, int R,
                                                 int RT, const double *__restrict__ W,
                                                 int pass, double *__restrict__ colsq,
                                                 const double *__restrict__ lambda,
                                                 FT *__restrict__ A)
{
    __shared__ double red[256];
    __shared__ double sW[32 * 32];
    __shared__ float sM[256];                  // RP * R <= 256 because RT >= R
    const int r = threadIdx.x % RT, g = threadIdx.x / RT, RP = 256 / RT;
    const bool wl = R <= 32;
    if (wl)
        for (int e = threadIdx.x; e < R * R; e += 256) sW[e] = W[e];
    __syncthreads();
    const double lam = (pass == 1 && r < R) ? lambda[r] : 1.0;
    double acc = 0.0;
    const int64_t per = (I + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per;
    const int64_t i1 = (i0 + per < I) ? i0 + per : I;
    if (wl) {                                    // uniform branch
        const bool on = r < R;
        const int base = (threadIdx.x & 63) - r; // lane of the row's element 0
        constexpr int U = 4;
        for (int64_t i = i0 + g; i < i1; i += (int64_t)U * RP) {
            float m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = i + (int64_t)u * RP;
                m[u] = (on && row < i1) ? M[row * R + r] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = i + (int64_t)u * RP;
                if (row >= i1) break;            // the row's lanes leave together
                double x = 0.0;
                for (int q = 0; q < R; ++q) {
                    const float mq = __shfl(m[u], base + q, 64);
                    const double w = on ? sW[q * R + r] : 0.0;
                    x += (double)mq * w;
                }
                if (on) {
                    if (pass == 0) acc += x * x;
                    else st<FT>(A, row * R + r, lam > 0.0 ? x / lam : x);
                }
            }
        }
    }
    for (int64_t ib = i0; !wl && ib < i1; ib += RP) {
        const int nrow = (int)((ib + RP < i1) ? RP : i1 - ib);
        for (int e = threadIdx.x; e < nrow * R; e += 256) sM[e] = M[ib * R + e];
        __syncthreads();
        if (r < R && g < nrow) {
            const float *m = sM + g * R;
            double x = 0.0;
            for (int q = 0; q < R; ++q) x += (double)m[q] * W[q * R + r];
            if (pass == 0) acc += x * x;
            else st<FT>(A, (ib + g) * R + r, lam > 0.0 ? x / lam : x);
        }
        __syncthreads();
    }
    if (pass == 0) {
        red[threadIdx.x] = acc;
        __syncthreads();
        if (g == 0 && r < R) {
            double s = 0.0;
            for (int k = 0; k < RP; ++k) s += red[k * RT + r];
            colsq[(int64_t)blockIdx.x * R + r] = s;
        }
    }
}

// Block-wide sum of part[b * stride] for b < count: thread t adds b = t,
// t + 256, ... in order, then a fixed tree.  Result valid in thread 0.
__device__ __forceinline__ double block_sum_strided(const double *__restrict__ part,
                                                    int64_t count, int64_t stride, double *red)
{
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < count; b += 256) s += part[b * stride];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// lambda_r = sqrt(sum_b colsq[b][r]); one block of 256 threads per column.
__global__ __launch_bounds__(256) void lambda_kernel(const double *__restrict__ colsq, int nb,
                                                     int R, double *__restrict__ lambda)
{
    __shared__ double red[256];
    const int r = blockIdx.x;
    const double s = block_sum_strided(colsq + r, nb, R, red);
    if (threadIdx.x == 0) lambda[r] = sqrt(s);
}

// inner[b][r] = sum over the block's rows of M(i,r) * A(i,r).
template <typename FT>
__global__ __launch_bounds__(256) void inner_partial(const float *__restrict__ M,
                                                     const FT *__restrict__ A, int64_t I, int R,
                                                     int RT, double *__restrict__ part)
{
    __shared__ double red[256];
    const int r = threadIdx.x % RT, g = threadIdx.x / RT, RP = 256 / RT;
    const int64_t per = (I + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per;
    const int64_t i1 = (i0 + per < I) ? i0 + per : I;
    double acc = 0.0;
    if (r < R)
        for (int64_t i = i0 + g; i < i1; i += RP) acc += (double)M[i * R + r] * ld<FT>(A, i * R + r);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (g == 0 && r < R) {
        double s = 0.0;
        for (int k = 0; k < RP; ++k) s += red[k * RT + r];
        part[(int64_t)blockIdx.x * R + r] = s;
    }
}

// fit = 1 - sqrt(max(0, xx - 2 <X,Xhat> + ||Xhat||^2)) / sqrt(xx), with
// <X,Xhat> = sum_r lambda_r inner_r and ||Xhat||^2 = lambda^T (hadamard_w G_w)
// lambda.  One block of 256 threads, fixed reduction order.
__global__ __launch_bounds__(256) void fit_kernel(const double *__restrict__ inner, int nb,
                                                  const double *__restrict__ G, int nmodes,
                                                  const double *__restrict__ lambda, int R,
                                                  const double *__restrict__ xx,
                                                  double *__restrict__ fit)
{
    __shared__ double red[256];
    double in = 0.0;
    for (int r = 0; r < R; ++r) in += lambda[r] * block_sum_strided(inner + r, nb, R, red);
    double acc = 0.0;
    for (int e = threadIdx.x; e < R * R; e += 256) {
        const int p = e / R, q = e % R;
        double h = 1.0;
        for (int w = 0; w < nmodes; ++w) h *= G[(int64_t)w * R * R + e];
        acc += lambda[p] * lambda[q] * h;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double res = xx[0] - 2.0 * in + red[0];
        fit[0] = 1.0 - sqrt(res > 0.0 ? res : 0.0) / sqrt(xx[0]);
    }
}

// Sum of squares of the record values (||X||^2), per-block partials.
__global__ __launch_bounds__(256) void sumsq_partial(const uint32_t *__restrict__ rec, int64_t nnz,
                                                     int NW, double *__restrict__ part)
{
    __shared__ double red[4];
    const int64_t per = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per;
    const int64_t i1 = (i0 + per < nnz) ? i0 + per : nnz;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double v = (double)__uint_as_float(rec[i * NW + NW - 1]);
        acc += v * v;
    }
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Clear n int32 counters (a kernel rather than a memset: safe to capture).
__global__ void zero_i32(int32_t *__restrict__ p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// out[0] = sum_b part[b] (one block of 256 threads, fixed order).
__global__ __launch_bounds__(256) void sum_kernel(const double *__restrict__ part, int64_t nb,
                                                  double *__restrict__ out)
{
    __shared__ double red[256];
    const double s = block_sum_strided(part, nb, 1, red);
    if (threadIdx.x == 0) out[0] = s;
}

}  // namespace als
