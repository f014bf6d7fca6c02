/*
 * mttkrp.h - C ABI of the MI355X (gfx950) all-mode sparse MTTKRP library.
 *
 * The library computes, for an N-mode sparse tensor X in coordinate (COO)
 * form and dense factor matrices A_0..A_{N-1} (each I_w x R, row-major),
 *
 *   M_n(i, r) = sum over nonzeros e with c_n(e) = i of
 *               val(e) * prod_{w != n} A_w(c_w(e), r)
 *
 * along every mode n (the elementwise spMTTKRP update of Sec. II-C and
 * Eq. 4 of Wijeratne, Kannan, Prasanna, "Dynasor", arXiv 2309.09131), with
 * the paper's dynamic tensor remapping (Sec. III-B): the nonzeros are kept
 * in one buffer ordered for the mode being computed and, once mode n is
 * computed (or during it, in the fused form), copied into the order of mode
 * (n+1) mod N (Alg. "Dynasor", dynamic remapping store), so that two
 * tensor-sized buffers serve all modes.  Around it: one CP-ALS sweep (Alg. "cp-als"), and the sampled CP
 * loss sum_e (x_e - sum_r prod_n A_n(c_n(e), r))^2 with its gradient.
 *
 * Conventions for every entry point
 *   - Pointers named d_* are HIP device pointers (device memory of the GPU
 *     that is current when the call is made); all others are host pointers.
 *   - The caller owns every device allocation (workspace, tensor, factors,
 *     outputs).  The library never allocates device memory; a plan owns
 *     only a small host object, HIP events and a non-blocking side stream
 *     of default priority (the reduction of rows split across shards runs
 *     there, ordered by events; every call makes `stream` wait for it).
 *   - `stream` is a hipStream_t passed as void* (NULL = legacy default
 *     stream).  Except mttkrp_plan (synchronous), calls only enqueue work
 *     on `stream` and return; a plan must be used by one stream at a time.
 *   - Factor matrices are row-major I_w x R, FP32 (MTTKRP_F32) or BF16
 *     (MTTKRP_BF16, stored bfloat16, widened to FP32 in registers).  MTTKRP
 *     outputs and gradients are FP32, row-major I_n x R.
 *   - Errors are status codes; nothing aborts or throws across the ABI.
 *     Argument errors are detected on the host before any device work.
 *   - Limits: 2 <= N <= 8, 1 <= R <= 256, 1 <= I_n < 2^31,
 *     0 <= nnz <= MTTKRP_MAX_NNZ (2^31 - 2^20).
 *   - Results are deterministic: no global atomics, fixed reduction order,
 *     so repeated calls give bit-identical outputs.
 */
#ifndef MTTKRP_H
#define MTTKRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTTKRP_MAX_MODES 8
#define MTTKRP_MAX_RANK 256
/* Largest nnz a plan accepts: 2^31 - 2^20.  Kernels index nonzeros with
 * 32-bit integers and form indices a few hundred past a shard's end before
 * clamping them, so the margin keeps every such index below 2^31. */
#define MTTKRP_MAX_NNZ 2146435072

typedef struct mttkrp_plan_s *mttkrp_plan_t;

typedef enum {
    MTTKRP_OK = 0,
    MTTKRP_EINVAL = 1,  /* bad argument (null pointer, size, mode, dtype) */
    MTTKRP_ERANGE = 2,  /* a coordinate is outside [0, I_n)               */
    MTTKRP_ENOMEM = 3,  /* workspace smaller than mttkrp_plan_workspace  */
    MTTKRP_ESTATE = 4,  /* tensor is in another mode's layout and the plan
                           was built with MTTKRP_NO_IMPLICIT_REMAP        */
    MTTKRP_EHIP = 5     /* a HIP call failed; see mttkrp_last_error      */
} mttkrp_status;

typedef enum { MTTKRP_F32 = 0, MTTKRP_BF16 = 1 } mttkrp_dtype;

/* flags */
#define MTTKRP_NO_IMPLICIT_REMAP 1u  /* mttkrp_mode on another layout fails  */
#define MTTKRP_NATURAL_ORDER 2u      /* dispatch shards in tensor order
                                        instead of longest-first order     */
#define MTTKRP_FUSED_REMAP 4u        /* write L_{n+1} from inside the MTTKRP
                                        kernel (the paper's same-agent remap)
                                        instead of a remap kernel right after
                                        it (default: measured faster here)  */
#define MTTKRP_UNPACKED_RECORDS 8u   /* one 32-bit word per stored
                                        coordinate instead of the default
                                        bit-packed form (see mttkrp_plan);
                                        for comparison                     */
#define MTTKRP_GATHER_ONLY 16u       /* measurement only: MTTKRP passes run a
                                        kernel that issues the MTTKRP kernel's
                                        record loads and factor-row gathers
                                        (same lanes, same row reuse) but adds
                                        every product into one register; the
                                        outputs are NOT MTTKRP results.  Its
                                        time bounds the MTTKRP kernel's from
                                        below for the same access stream.
                                        Needs the contiguous lane forms (R a
                                        multiple of 4 for FP32, 8 for BF16). */

#define MTTKRP_LOCALITY_ORDER 32u    /* plan option (Sec. V-J, Z-Morton
                                        ordering at preprocessing): inside
                                        each output row of L_n the nonzeros
                                        follow the Morton code of their two
                                        leading inputs (c_{n-1}, c_{n-2};
                                        c_{n-1} the more significant), then
                                        c_{n-3}, ..., c_{n+1}, then input
                                        position, instead of the cyclic
                                        lexicographic order; P_n is composed
                                        from the two layouts.  Results are the
                                        same sums in another order.         */

/* Memory for time (plan option): keep a copy of the layout L_n resident in
 * the workspace for every mode n whose bit is set (bits 16 + n).  Moving to
 * a resident layout then switches buffers instead of running the remap into
 * it; results and layouts are unchanged.  Each resident layout costs nnz
 * stored records of workspace beyond the paper's two buffers (Sec. IV-B);
 * keeping every mode's layout is the paper's "without dynamic remapping"
 * case (Sec. V).  EINVAL for a bit at or above nmodes. */
#define MTTKRP_RESIDENT_LAYOUT(n) (1u << (16 + (n)))

/* Partitioning parameters (Sec. III-A, III-C).  Zero selects a default. */
typedef struct {
    int32_t g;                       /* nonzeros per shard; default 1024     */
    int32_t m[MTTKRP_MAX_MODES];     /* indices per super-shard, per mode:
                                        default follows Sec. V-A: 1 when
                                        I_n < workers, else I_n / (q*workers)
                                        kept in (1000, 16000) when possible  */
    int32_t workers;                 /* nu: scheduling bins; default 256     */
    uint32_t flags;
} mttkrp_plan_opts;

/* Bytes of device workspace a plan needs (ws_bytes for mttkrp_plan).
 * Layout-independent upper bound; depends on N, dims, nnz, rank, opts. */
mttkrp_status mttkrp_plan_workspace(int nmodes, const int64_t *dims, int64_t nnz,
                                    int rank, const mttkrp_plan_opts *opts,
                                    size_t *bytes);

/*
 * Preprocess a COO tensor (Sec. III-A partitions, Sec. V-J preprocessing).
 *   d_idx   [nmodes][nnz] int32, mode-major, 0-based coordinates.
 *   d_vals  [nnz] float values.  Duplicated coordinates are accepted and
 *           summed by every MTTKRP.
 * Builds, inside d_workspace: the mode-0 layout L_0 (nonzeros ordered by
 * (c_0, c_{N-1}, ..., c_1, input position)), for every mode n the remap
 * target P_n (slot of each L_n element in L_{n+1}), row pointers, the
 * super-shard / shard tables and the longest-first schedule (Alg.
 * "ss_scheduling"), and per layout the tables that give the output row of
 * any position.  The inputs are copied; they may be freed afterwards.
 * A stored nonzero record of layout L_m holds the N-1 coordinates other
 * than c_m, which its position implies (L_m is ordered by c_m first),
 * bit-packed (b_n = bit length of I_n - 1 bits each, in mode order, in as
 * few 32-bit words as the compiled widths allow for the widest layout: at
 * least 2 words at four modes, N-3 from five modes on) followed by the FP32
 * value; MTTKRP_UNPACKED_RECORDS stores one word per stored coordinate.
 * The remap L_n -> L_{n+1} stores c_n in each record it moves and drops
 * c_{n+1}.
 * The workspace must stay allocated and untouched while the plan lives.
 * Synchronous: returns after the device work finished.  ERANGE if a
 * coordinate is out of range (nothing else is then valid).
 */
mttkrp_status mttkrp_plan(int nmodes, const int64_t *dims, int64_t nnz,
                          const int32_t *d_idx, const float *d_vals, int rank,
                          const mttkrp_plan_opts *opts, void *d_workspace,
                          size_t ws_bytes, void *stream, mttkrp_plan_t *out);

/*
 * MTTKRP along one mode (Eq. 4).  d_factors: host array of nmodes device
 * pointers (the output mode's factor is read only by cp_loss_grad and may
 * be NULL here).  d_out: I_mode x R FP32, fully overwritten (rows without
 * nonzeros become +0.0).  If the tensor is not in L_mode it is first
 * remapped forward (ESTATE instead under MTTKRP_NO_IMPLICIT_REMAP).
 * fuse_remap != 0 also remaps the tensor to L_{mode+1} (Sec. III-B) and
 * leaves the plan there: by a remap kernel enqueued right after the MTTKRP,
 * or inside the MTTKRP pass itself (Sec. V-B, same agent) when the plan was
 * built with MTTKRP_FUSED_REMAP.
 */
mttkrp_status mttkrp_mode(mttkrp_plan_t p, int mode, const void *const *d_factors,
                          mttkrp_dtype fdt, float *d_out, int fuse_remap,
                          void *stream);

/* MTTKRP along all modes n = 0..N-1, each followed by the remap into the
 * next mode's layout (Alg. "Dynasor"); every mode uses the given factors.
 * d_out: host array of nmodes device pointers, each I_n x R FP32.  The
 * buffers may overlap (even be one buffer): a pass that writes memory still
 * being written by an earlier pass waits for it, so each buffer ends up
 * with the result of the last mode written into it.  Starts from L_0
 * (remapping first if needed) and ends in L_0. */
mttkrp_status mttkrp_all_modes(mttkrp_plan_t p, const void *const *d_factors,
                               mttkrp_dtype fdt, float *const *d_out,
                               void *stream);

/* Standalone remapping (Sec. III-B): advance the layout L_cur -> L_cur+1 ->
 * ... -> L_to_mode.  No-op when already there. */
mttkrp_status remap(mttkrp_plan_t p, int to_mode, void *stream);

/*
 * Sampled CP loss L = sum_e (x_e - m_e)^2, m_e = sum_r prod_n A_n(c_n(e), r)
 * (the CP model of Eq. 1 evaluated at the stored nonzeros; no 1/2, no
 * mean), and optionally its gradient
 *   dL/dA_k(i, r) = -2 * s * sum_{e: c_k(e) = i} rho_e prod_{n != k} A_n(c_n(e), r)
 * with rho_e = x_e - m_e recomputed per pass (never stored) and s the
 * scale *d_grad_scale (NULL: 1.0; a device double, e.g. the upstream
 * gradient of an autograd graph).
 *   d_loss   device double or NULL.
 *   d_grads  host array of nmodes device pointers (I_k x R FP32) or NULL.
 * With gradients: N residual-MTTKRP passes with fused remap, ending in the
 * layout it started in; with the loss as well, the first of them also sums
 * the squared residuals (the same FP32 terms, FP64 accumulation and
 * reduction order as the loss-only pass, so the same value), except under
 * MTTKRP_FUSED_REMAP, which runs the loss pass first.  Loss only: one pass,
 * layout unchanged.
 */
mttkrp_status cp_loss_grad(mttkrp_plan_t p, const void *const *d_factors,
                           mttkrp_dtype fdt, double *d_loss, float *const *d_grads,
                           const double *d_grad_scale, void *stream);

/*
 * One CP-ALS sweep (Alg. "cp-als"), Gauss-Seidel over n = 0..N-1:
 *   M_n = MTTKRP(n) with fused remap; V = hadamard_{w != n} A_w^T A_w;
 *   A_n = M_n V^{-1} (Cholesky, FP64); lambda_r = ||A_n(:, r)||_2,
 *   A_n(:, r) /= lambda_r (zero columns left as is); store A_n in fdt
 *   (BF16: round to nearest even); G_n = A_n^T A_n of the stored values.
 * Gram matrices, Cholesky, solve and the norm / fit reductions run in FP64.
 *   d_factors  in/out, host array of nmodes device pointers (fdt).
 *   d_mbuf     FP32 scratch of max_n I_n x R elements.
 *   d_lambda   device double[R], lambda of the last mode.
 *   d_fit      device double or NULL: 1 - ||X - Xhat||_F / ||X||_F.
 * If a Cholesky factorisation fails, 1e-12 * trace(V) / R is added to the
 * diagonal once (counted in the MTTKRP_INFO_RIDGE info after a sync).
 */
mttkrp_status cp_als_sweep(mttkrp_plan_t p, void *const *d_factors,
                           mttkrp_dtype fdt, float *d_mbuf, double *d_lambda,
                           double *d_fit, void *stream);

/*
 * The CP-ALS sweep of cp_als_sweep without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The FP32 scratch that
 * cp_als_sweep takes as d_mbuf is instead a static device array of
 * MTTKRP_STATIC_MBUF_FLOATS floats (64 MiB) inside the library; every GPU
 * the library runs on holds its own copy until the process ends.  The call
 * allocates nothing and creates no HIP objects: the plan made its stream
 * and events when it was built, and kernel timing (mttkrp_profile) is not
 * applied to this call's launches.  Results equal cp_als_sweep's.
 *   EINVAL if max_n I_n * R > MTTKRP_STATIC_MBUF_FLOATS (before any work).
 * All calls on one GPU share the array, and each leaves its contents behind
 * (every MTTKRP output is fully written before it is read, so nothing needs
 * clearing).  Calls that overlap in time on one GPU -- from different
 * streams, threads or plans -- race on the array; calls on one stream are
 * ordered.  Other arguments as in cp_als_sweep.
 */
#define MTTKRP_STATIC_MBUF_FLOATS 16777216
mttkrp_status cp_als_sweep_static(mttkrp_plan_t p, void *const *d_factors,
                                  mttkrp_dtype fdt, double *d_lambda, double *d_fit,
                                  void *stream);

/*
 * CP-ALS to convergence (Alg. "cp-als" with its loop): sweeps as in
 * cp_als_sweep until two consecutive fits differ by less than tol, or
 * max_sweeps sweeps.  The Gram matrices are computed once at the start and
 * then kept current (each mode update refreshes its own), not recomputed
 * every sweep; the results equal max_sweeps calls of cp_als_sweep.
 * Synchronises `stream` after every sweep to read the fit.  The fit comes
 * from ||X||^2 - 2<X, Xhat> + ||Xhat||^2 with FP32 MTTKRP values, so near
 * an exact fit it carries noise of about 1e-4: tolerances below that may
 * never be met there (1e-4 is the usual CP-ALS default).
 *   max_sweeps   >= 1;  tol >= 0 (0: run max_sweeps sweeps).
 *   d_fit_trace  device double[max_sweeps] or NULL: the fit after each sweep.
 *   sweeps, fit  host out (nullable): sweeps run and the last fit.
 * Other arguments as in cp_als_sweep.
 */
mttkrp_status cp_als(mttkrp_plan_t p, void *const *d_factors, mttkrp_dtype fdt,
                     float *d_mbuf, double *d_lambda, int max_sweeps, double tol,
                     double *d_fit_trace, int *sweeps, double *fit, void *stream);

/* Device-side plan arrays, copied into caller memory (for parity tests). */
enum {
    MTTKRP_Q_LAYOUT = 0,   /* current element buffer, widened to
                              nnz x (N int32 + f32)                          */
    MTTKRP_Q_PERM = 1,     /* P_mode: nnz int32                              */
    MTTKRP_Q_ROW_PTR = 2,  /* I_mode + 1 int32                               */
    MTTKRP_Q_SHARDS = 3,   /* nshards x {start, len, super-shard} int32      */
    MTTKRP_Q_LPT = 4       /* k_mode int32: scheduling bin of each super-shard */
};
/* Copies the array `what` of `mode` into dst (device or host memory,
 * hipMemcpyDefault; synchronises `stream`).  Sizes in bytes: LAYOUT
 * nnz*(N+1)*4 (the layout the tensor is currently in, its stored records
 * widened on the host to one int32 per coordinate, the layout's own
 * coordinate taken from its row pointers), PERM nnz*4, ROW_PTR
 * (I_mode+1)*4, SHARDS nshards*12, LPT k_mode*4.  EINVAL if bytes is
 * smaller. */
mttkrp_status mttkrp_plan_query(mttkrp_plan_t p, int what, int mode, void *dst,
                                size_t bytes, void *stream);

/* Host-side scalars. */
enum {
    MTTKRP_INFO_CUR_MODE = 0,     /* layout the tensor is in                 */
    MTTKRP_INFO_NSHARDS = 1,      /* shards of `mode`                        */
    MTTKRP_INFO_NSUPER = 2,       /* super-shards of `mode` (k_n)            */
    /* 3: reserved */
    MTTKRP_INFO_NSPLIT = 4,       /* rows of `mode` split across shards      */
    MTTKRP_INFO_G = 5,            /* shard size used                         */
    MTTKRP_INFO_M = 6,            /* super-shard size of `mode`              */
    MTTKRP_INFO_RIDGE = 7,        /* ridge count of the last cp_als_sweep
                                     (reads device memory; synchronises)    */
    MTTKRP_INFO_RECORD_BYTES = 8  /* bytes of one stored nonzero record     */
};
mttkrp_status mttkrp_plan_info(mttkrp_plan_t p, int what, int mode, int64_t *value);

/* Kernel timing with HIP events on the launch stream: when enabled, every
 * launch of the per-mode MTTKRP kernel, the remap kernel, the residual
 * (loss-gradient) MTTKRP kernel and the loss kernel is bracketed by events.
 * mttkrp_profile_read synchronises and returns the summed milliseconds and
 * launch count of `kernel` (one of the MTTKRP_PROF_* ids) for `mode` (-1:
 * all modes; for the remap kernel, the mode it remaps from; the loss kernel
 * runs on the layout of its mode) since the last read, and resets those
 * events. */
#define MTTKRP_PROF_MTTKRP 0
#define MTTKRP_PROF_REMAP 1
#define MTTKRP_PROF_RESID 2
#define MTTKRP_PROF_LOSS 3
mttkrp_status mttkrp_profile(mttkrp_plan_t p, int enable);
mttkrp_status mttkrp_profile_read(mttkrp_plan_t p, int kernel, int mode, double *ms,
                                  int64_t *launches);

/* Frees the host object (never the caller's workspace). */
mttkrp_status mttkrp_plan_destroy(mttkrp_plan_t p);

const char *mttkrp_status_str(mttkrp_status st);
/* Text of the last error on `p` (or of the last plan-less error when p is
 * NULL); valid until the next call on the same plan. */
const char *mttkrp_last_error(mttkrp_plan_t p);

#ifdef __cplusplus
}
#endif
#endif /* MTTKRP_H */
