/*
 * libmttkrp -- dense 3-way MTTKRP and CP-ALS on AMD Instinct MI355X (gfx950).
 *
 * What is computed.  For a dense tensor X of shape I x J x K (row-major,
 * element (i,j,k) at offset (i*J + j)*K + k) and factor matrices
 * A (I x R), B (J x R), C (K x R) (row-major, r fastest), the mode-n MTTKRP
 * (matricised tensor times Khatri-Rao product) is
 *
 *     mode 0:  M(i,r) = sum_{j,k} X(i,j,k) B(j,r) C(k,r)      (I x R)
 *     mode 1:  M(j,r) = sum_{i,k} X(i,j,k) A(i,r) C(k,r)      (J x R)
 *     mode 2:  M(k,r) = sum_{i,j} X(i,j,k) A(i,r) B(j,r)      (K x R)
 *
 * i.e. M_n = X_(n) times the Khatri-Rao product of the other two factors.
 * CP-ALS updates each factor from its normal equations A_n V = M_n with
 * V = Hadamard product of the other two Gram matrices A_m^T A_m, then
 * normalises its columns to unit 2-norm (the norms become lambda).  The
 * paper this library accompanies (arXiv 2411.04785) has no passage on these
 * operations; the definitions above are the standard ones.
 *
 * Conventions for every entry point:
 *  - Data pointers are DEVICE pointers owned by the caller.  The library
 *    never frees, reallocates or retains them after the call returns, except
 *    inside the als_sweep graph cache (released by mtk_graph_reset or
 *    mtk_destroy).  `fit_host` in als_sweep is the only host buffer.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously on it; arguments are validated synchronously.
 *  - Invalid arguments return MTK_EINVAL with a message in mtk_last_error
 *    and enqueue nothing.  Errors detected on the device (a non-positive
 *    elimination pivot) set a sticky status word that mtk_check returns.
 *  - NaN / Inf inputs propagate to the outputs; they are not checked.
 *  - A context is not thread-safe: use one per host thread.  All entry
 *    points of one context must use the same device.
 *  - The library never throws across the ABI.
 */
#ifndef MTTKRP_H_
#define MTTKRP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mtk_ctx mtk_ctx;

typedef enum {
  MTK_OK = 0,
  MTK_EINVAL = -1,        /* invalid argument (nothing was enqueued) */
  MTK_ENOMEM = -2,        /* device allocation failed */
  MTK_EHIP = -3,          /* a HIP runtime call failed (message in mtk_last_error) */
  MTK_ENOTSPD = -4,       /* normal-equation matrix not positive definite */
  MTK_EUNSUPPORTED = -5,  /* valid but unsupported combination */
  MTK_EBUDGET = -6,       /* serving: request larger than the whole HBM budget */
  MTK_EAGAIN = -7         /* serving: nothing finished yet */
} mtk_status;

/* Arithmetic of the contraction.  All paths accumulate in FP32.
 *  MTK_FP32     : FP32 products (FP32 MFMA).
 *  MTK_BF16X3   : each FP32 operand split into bf16 hi = bf16(x) and
 *                 lo = bf16(x - hi); the product is hi*hi + hi*lo + lo*hi
 *                 on bf16 MFMA (the lo*lo term, below 2^-16 relative, is
 *                 dropped).
 *  MTK_BF16X6   : each FP32 operand split into three bf16 terms hi = bf16(x),
 *                 mid = bf16(x - hi), lo = bf16(x - hi - mid) (together the
 *                 24 significand bits of x); the six products down to 2^-16
 *                 relative (lo*hi, hi*lo, mid*mid, mid*hi, hi*mid, hi*hi) on
 *                 bf16 MFMA; what is dropped is below 2^-24, so the error
 *                 is that of FP32 accumulation.  FP32 tensors; not served.
 *  MTK_FP8_E4M3 : OCP e4m3 tensor with per mode-1 slice power-of-two scales
 *                 (see mtk_quantize_fp8) on e4m3 MFMA; the factor inside the
 *                 contraction is held as two e4m3 terms, hi = e4m3(g 2^-eh)
 *                 and lo = e4m3((g - hi 2^eh) 2^-el), with power-of-two
 *                 scales eh, el per column (about 2^-8 relative). */
typedef enum { MTK_FP32 = 0, MTK_BF16X3 = 1, MTK_FP8_E4M3 = 2, MTK_BF16X6 = 3 } mtk_prec;

/* Dense tensor descriptor.
 *  data      : device pointer; FP32 values (fmt MTK_FP32) or e4m3 codes, one
 *              byte each (fmt MTK_FP8_E4M3), row-major (i, j, k), k fastest.
 *  data_t    : FP8 only, optional (may be NULL): the same codes with every
 *              mode-1 slice transposed, element (i,j,k) at (i*K + k)*J + j
 *              (see mtk_quantize_fp8).  When present, mode 2 reads it.
 *  dims      : I, J, K (each >= 1, I*J*K < 2^40).
 *  fmt       : MTK_FP32 or MTK_FP8_E4M3.
 *  slice_exp : FP8 only: device int32[I]; the value of element (i,j,k) is
 *              decode(code) * 2^slice_exp[i].  NULL for FP32.  */
typedef struct {
  const void* data;
  const void* data_t;
  int64_t dims[3];
  int32_t fmt;
  const int32_t* slice_exp;
} mtk_tensor;

/* Create a context on HIP device `device` (makes it current).  The context
 * owns a workspace that grows on demand and a sticky device status word.
 * Growing the workspace allocates a larger block without waiting for the
 * device; the outgrown block is kept until mtk_graph_reset or mtk_destroy. */
mtk_status mtk_create(mtk_ctx** ctx, int device);

/* Destroy a context, its workspace and its graph cache.  NULL is a no-op. */
mtk_status mtk_destroy(mtk_ctx* ctx);

/* Message of the last failing call on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char* mtk_last_error(const mtk_ctx* ctx);

/* Synchronise `stream`, then return and clear the sticky device status:
 * MTK_OK, or MTK_ENOTSPD if an elimination pivot of V was <= 0 since the
 * last check (V is then not positive definite). */
mtk_status mtk_check(mtk_ctx* ctx, void* stream);

/* Reserve workspace for MTTKRPs / solves / sweeps up to these sizes, so
 * later calls of at most this size allocate nothing.  Optional. */
mtk_status mtk_reserve(mtk_ctx* ctx, const int64_t dims[3], int64_t R, int prec);

/* FP8 tensor preparation (operand prep).  x: FP32 tensor of shape dims
 * (device).  For each mode-1 slice i, e_i = min{ e : amax_i <= 448 * 2^e }
 * (0 for an all-zero slice; e_i is kept within [-126, 119]) is written to
 * exp_out[i] and q_out = e4m3(x * 2^-e_i) with round-to-nearest-even,
 * saturating to +-448, the sign kept for values that round to zero,
 * NaN -> 0x7F.  q_out holds I*J*K bytes in the same order as x.  If qt_out
 * is not NULL it receives the same codes with each slice transposed
 * (element (i,j,k) at (i*K + k)*J + j), the layout mtk_tensor.data_t takes.
 * Bit-exact and deterministic. */
mtk_status mtk_quantize_fp8(mtk_ctx* ctx, const float* x, const int64_t dims[3],
                            uint8_t* q_out, uint8_t* qt_out, int32_t* exp_out, void* stream);

/* Mode-n MTTKRP (see top of file).
 *  X        : tensor descriptor (device data).
 *  factors  : host array of three device pointers A, B, C (FP32, row-major,
 *             dims[n] x R).  factors[mode] is not read and may be NULL.
 *  R        : 1 <= R <= 128.
 *  mode     : 0, 1 or 2.
 *  prec     : MTK_FP32, MTK_BF16X3 or MTK_BF16X6 for an FP32 tensor; MTK_FP8_E4M3 for
 *             an FP8 tensor (the tensor's fmt decides; prec must match).
 *  out      : device FP32, dims[mode] x R row-major; fully overwritten.
 * The result is deterministic: the summation order depends only on
 * (dims, R, mode, prec), never on timing or on other work on the device.
 * (bf16x3 mode 0 with J a multiple of 256 -- 128 above R = 64 --,
 * K >= 512 and J*K >= 65536 is formed as mttkrp_dimtree's mode 0, bit for
 * bit.) */
mtk_status mttkrp(mtk_ctx* ctx, const mtk_tensor* X, const float* const factors[3],
                  int64_t R, int mode, int prec, float* out, void* stream);

/* mttkrp without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels, plan and result (bit for bit)
 * as mttkrp; the caller passes X, the factors and out as before.  The
 * split-K partial slices (for bf16x3 mode 0 as above, the J-block partial
 * rows) and FP8 fragment codes go to a static device
 * buffer of 64 MiB (one per device, held from library load until the
 * process ends) instead of the context's workspace, and the call makes no
 * hipMalloc, hipFree or other allocating call.  Nothing in the buffer needs
 * to start at zero (every byte a launch reads it has written first).
 * Every call on one device shares that device's buffer: calls that overlap
 * on one device (any stream, any context) race and must be serialised by
 * the caller.  Returns MTK_EUNSUPPORTED, enqueueing nothing, for a shape
 * whose plan needs more than 64 MiB of scratch (large outputs at high rank,
 * e.g. 2048^3 at R = 128). */
mtk_status mttkrp_noalloc(mtk_ctx* ctx, const mtk_tensor* X, const float* const factors[3],
                          int64_t R, int mode, int prec, float* out, void* stream);

/* Mode-n MTTKRP of a dense N-way tensor (3 <= N <= 8), FP32 in memory:
 *     M(i_n, r) = sum over all other indices of X(i_1, ..., i_N)
 *                 * prod_{m != n} A_m(i_m, r)
 * (the tensor unfolded along mode n times the Khatri-Rao product of the
 * other N-1 factors; the standard definition, which the paper does not
 * state).  The row-major bytes of X are viewed as a three-way tensor that
 * merges consecutive modes -- (P, d_n, Q) for a middle mode, with the first
 * and last modes splitting the others into two groups of balanced size --
 * and a merged group's factor is the Khatri-Rao product of its factors
 * (first mode's index slowest), formed in FP32 in the context's workspace;
 * the three-way contraction then runs as mttkrp does.  With N = 3 the result
 * is mttkrp's, bit for bit.
 *  X       : device FP32, element (i_1..i_N) at ((i_1 d_2 + i_2) d_3 + ...) .
 *  dims    : host int64[nmodes], each >= 1, product < 2^40, and every merged
 *            group's product <= 2^30 (else MTK_EUNSUPPORTED).
 *  factors : host array of nmodes device pointers (dims[m] x R, FP32,
 *            row-major); factors[mode] is not read and may be NULL.
 *  prec    : MTK_FP32, MTK_BF16X3 or MTK_BF16X6.
 *  R, mode, out, stream : as for mttkrp (out is dims[mode] x R). */
mtk_status mttkrp_nway(mtk_ctx* ctx, const float* X, int nmodes, const int64_t* dims,
                       const float* const* factors, int64_t R, int mode, int prec, float* out,
                       void* stream);

/* Sparse three-way tensors in coordinate form.
 *
 * A sparse tensor is a list of nnz stored entries (i, j, k, v); repeated
 * coordinates add.  Its mode-n MTTKRP is the dense definition above with the
 * sum restricted to the stored entries, e.g. for mode 0
 *     M(i,r) = sum over entries (i, j, k, v) of v B(j,r) C(k,r)
 * (the standard definition; the paper has no passage on sparse tensors). */
typedef struct mtk_coo mtk_coo;

/* Copy the entries to the device in the library's form: for each mode, the
 * entries sorted by that mode's index (stable, so entries with equal index
 * keep their input order), 16 bytes each, plus the carry slots mttkrp_coo
 * uses -- about 48 bytes per entry in one allocation, freed by
 * mtk_coo_destroy.  The sort runs on `stream`, which is synchronised before
 * the call returns; the caller's arrays may be freed afterwards.
 *  dims   : host int64[3], each in [1, 2^31 - 1].
 *  nnz    : number of entries, 0 <= nnz < 2^31.
 *  idx    : host array of three device int32 arrays (nnz each, 4-byte
 *           aligned): the i, j and k index of every entry.
 *  vals   : device FP32[nnz] values.
 *  out    : receives the handle (NULL on failure).
 * MTK_EINVAL (nothing kept) if an index lies outside dims; MTK_ENOMEM if the
 * device allocation fails. */
mtk_status mtk_coo_create(mtk_ctx* ctx, const int64_t dims[3], int64_t nnz, const int32_t* const idx[3],
                          const float* vals, void* stream, mtk_coo** out);
/* Free a tensor made by mtk_coo_create (synchronises its device).  NULL is a no-op. */
mtk_status mtk_coo_destroy(mtk_coo* t);
/* Number of stored entries of t, or -1 for NULL. */
int64_t mtk_coo_nnz(const mtk_coo* t);

/* Mode-n MTTKRP of a sparse tensor, FP32 products and sums.  Each output row
 * is the sum of its entries' terms in entry order (the sorted order), cut
 * into segments of a length that depends on nnz only, the segments' partial
 * sums then added in order: the result is deterministic.
 *  factors : the two factors other than `mode` are read (device FP32,
 *            dims[m] x R row-major); factors[mode] may be NULL.
 *  R       : 1..128.  out : device FP32, dims[mode] x R, overwritten.
 * Calls on one mtk_coo must not overlap in time (they share its carry
 * slots); calls on different tensors may. */
mtk_status mttkrp_coo(mtk_ctx* ctx, const mtk_coo* t, const float* const factors[3], int64_t R, int mode,
                      float* out, void* stream);

/* CP-ALS sweeps on a sparse tensor: for modes 0, 1, 2 in order, mttkrp_coo
 * into factors[mode] and gram_solve in place (the dense sweep's update,
 * unchanged).  lambda (device FP64[R]) is overwritten; the factors given
 * are the starting point.  Synchronises `stream` at the end and returns the
 * sticky status (MTK_OK or MTK_ENOTSPD, see mtk_check).  MTK_EUNSUPPORTED
 * if a dimension exceeds 2^30 (the update's limit). */
mtk_status als_sweep_coo(mtk_ctx* ctx, const mtk_coo* t, float* const factors[3], double* lambda, int64_t R,
                         int nsweeps, void* stream);

/* CP-ALS sweeps of an N-way tensor (3 <= N <= 8): each sweep updates the
 * factors in mode order, A_n = M_n V^{-1} with M_n the mode-n MTTKRP (as
 * mttkrp_nway computes it) and V the Hadamard product of the Gram matrices
 * of the other N-1 factors, then normalises A_n's columns into lambda.  In
 * the three-way view of mode n the merged groups' factors are their
 * Khatri-Rao products, whose Gram matrices are the Hadamard products of
 * their factors' Grams, so each update is gram_solve on that view.  The
 * standard CP-ALS (the paper has no passage on it).
 *  X, nmodes, dims, R, prec : as for mttkrp_nway (every merged dimension
 *          <= 2^30, else MTK_EUNSUPPORTED).
 *  factors : host array of nmodes device pointers (dims[m] x R FP32), the
 *            starting point, updated in place.
 *  lambda  : device FP64[R], overwritten.
 * Synchronises `stream` at the end and returns the sticky status (MTK_OK or
 * MTK_ENOTSPD, see mtk_check). */
mtk_status als_sweep_nway(mtk_ctx* ctx, const float* X, int nmodes, const int64_t* dims, float* const* factors,
                          double* lambda, int64_t R, int prec, int nsweeps, void* stream);

/* Mode-0 or mode-1 MTTKRP by the dimension tree, the form als_sweep uses
 * for those two updates when mtk_sweep_uses_dimtree says so.  First
 * Y = X x_3 C, Y(i,j,r) = sum_k X(i,j,k) C(k,r) (an I*J x R FP32
 * intermediate in the context's workspace, one pass over X), then
 *     mode 0:  M(i,r) = sum_j Y(i,j,r) B(j,r)
 *     mode 1:  M(j,r) = sum_i Y(i,j,r) A(i,r)
 * which is the mttkrp result with its sums associated differently (equal up
 * to rounding).  Deterministic, and bitwise equal to the MTTKRP of the same
 * mode inside an als_sweep that uses the tree.
 *  X     : FP32 tensor, prec MTK_FP32, MTK_BF16X3 or MTK_BF16X6 (arithmetic of the
 *          contraction with C; the sums over Y are FP32).
 *  mode  : 0 or 1.  factors[2] and factors[1 - mode] are read.
 *  R, out, stream : as for mttkrp.
 * MTK_EUNSUPPORTED if dims[0]*dims[1] > 2^36. */
mtk_status mttkrp_dimtree(mtk_ctx* ctx, const mtk_tensor* X, const float* const factors[3],
                          int64_t R, int mode, int prec, float* out, void* stream);

/* 1 if als_sweep forms the mode-0 and mode-1 MTTKRPs of each sweep of this
 * shape, rank and precision by the dimension tree (two passes over X per
 * sweep instead of three), else 0.  Currently: FP32 tensors (MTK_FP32,
 * MTK_BF16X3) with dims[2] >= 8 R, where writing and twice reading Y costs
 * well under the pass it saves. */
int mtk_sweep_uses_dimtree(const int64_t dims[3], int64_t R, int prec);

/* Normal-equation update of one factor (FP64 on the device).
 *  V = *_{m != mode} A_m^T A_m  (R x R, FP64, from the FP32 factors)
 *  V^{-1} by symmetric elimination: the LDL^T (square-root-free Cholesky)
 *  factorisation of V carried out in Gauss-Jordan form, which also clears
 *  above the diagonal and so leaves V^{-1}; F = M V^{-1} (all FP64)
 *  lambda_out[r] = ||F(:,r)||_2 (FP64); factor_out = F(:,r)/lambda_r cast
 *  to FP32 (a column with lambda_r == 0 is written unscaled).
 *  factors    : three device pointers (factors[mode] not read, may be NULL).
 *  dims       : host int64[3], each in [1, 2^30] (no limit on the product:
 *               the update never touches the tensor).
 *  R          : 1..128.
 *  M          : device FP32 dims[mode] x R (an MTTKRP result).
 *  factor_out : device FP32 dims[mode] x R; may alias factors[mode] or M.
 *  lambda_out : device FP64[R].
 * A pivot <= 0 sets MTK_ENOTSPD in the sticky status (see mtk_check); the
 * outputs are then unspecified. */
mtk_status gram_solve(mtk_ctx* ctx, const float* const factors[3], const int64_t dims[3],
                      int64_t R, int mode, const float* M, float* factor_out,
                      double* lambda_out, void* stream);

/* Fit of a CP model: fit = 1 - ||X - [[lambda; A,B,C]]||_F / ||X||_F,
 * from the explicit residual accumulated in FP64 on the device.  Writes the
 * fit to *fit_host after synchronising the stream. */
mtk_status mtk_fit(mtk_ctx* ctx, const mtk_tensor* X, const float* const factors[3],
                   const double* lambda, int64_t R, double* fit_host, void* stream);

/* CP-ALS sweeps.  Each sweep updates modes 0, 1, 2 in order: mttkrp (for
 * modes 0 and 1 mttkrp_dimtree when mtk_sweep_uses_dimtree), then
 * gram_solve in place into factors[mode] and lambda.  The factors given are
 * used as the starting point (not normalised first); lambda (device FP64[R])
 * is overwritten.  Calling again with the same buffers continues the
 * iteration (10 sweeps == 5 + 5 sweeps, bitwise).  The sweep sequence is
 * captured once into a HIP graph per (shape, R, prec, pointers, stream) and
 * replayed.  If fit_host is not NULL, fit_host[s] receives the fit after
 * sweep s (an extra residual pass per sweep).  Synchronises `stream` once
 * at the end and returns the sticky status (MTK_OK or MTK_ENOTSPD). */
mtk_status als_sweep(mtk_ctx* ctx, const mtk_tensor* X, float* const factors[3],
                     double* lambda, int64_t R, int prec, int nsweeps, double* fit_host,
                     void* stream);

/* CP-ALS until the fit settles: up to max_sweeps sweeps (the same captured
 * sweep as als_sweep, so k sweeps here leave the factors bitwise equal to
 * als_sweep with nsweeps = k), stopping after the first sweep s >= 1 whose
 * fit differs from sweep s-1's by less than tol (tol = 0: run all).
 * The per-sweep fit costs no pass over X: at the least-squares solution of
 * the sweep's last update F = M V^{-1} (before normalising),
 * ||Xhat||^2 = <X, Xhat> = <F, M>, so
 *     fit = 1 - sqrt(max(0, ||X||^2 - <F, M>)) / ||X||
 * with <F, M> accumulated in FP64 by the update and ||X||^2 formed once per
 * call (one pass over X).  Its absolute error is about
 * e ||X|| / (2 ||X - Xhat||) for a relative MTTKRP error e (1e-7 FP32), so
 * it is a monitor, not the reported fit, at fits close to 1.
 *  fits_host   : host double[max_sweeps] or NULL; receives the per-sweep fits.
 *  sweeps_done : host int, sweeps run.
 *  fit_final   : host double or NULL; the direct-residual fit (as mtk_fit) of
 *                the final model.
 * Synchronises `stream` once per sweep.  Returns the sticky status; a
 * sweep that sets MTK_ENOTSPD ends the run. */
mtk_status als_run(mtk_ctx* ctx, const mtk_tensor* X, float* const factors[3], double* lambda,
                   int64_t R, int prec, int max_sweeps, double tol, double* fits_host,
                   int* sweeps_done, double* fit_final, void* stream);

/* als_run with an extrapolation step after every sweep s >= ls_start
 * (sweeps of this call counted from 1; ls_start >= 1).  After sweep s has
 * taken the first two factors from A_p, B_p to A_s, B_s, a candidate moves
 * them further along that change,
 *     A_E = normalise(A_p + d (A_s - A_p)),  B_E = normalise(B_p + d (B_s - B_p)),
 * d = s^(1/3), and solves the third factor exactly from A_E and B_E (one
 * more mode-2 MTTKRP and update).  The candidate replaces the sweep's
 * factors and lambda when its fit (from <F, M>, as for the per-sweep fit)
 * is higher.  The standard line search by extrapolation for CP-ALS (the
 * paper has no passage on it); a swamp of nearly collinear components is
 * where it pays.  Each sweep from ls_start on costs one more pass over X.
 *  fits_host     : NULL or host double[max_sweeps]: the fit kept after each sweep.
 *  accepted_host : NULL or host int[max_sweeps]: 1 where the candidate was kept.
 * Other arguments and the return value as for als_run. */
mtk_status als_run_extrapolated(mtk_ctx* ctx, const mtk_tensor* X, float* const factors[3], double* lambda,
                                int64_t R, int prec, int max_sweeps, double tol, int ls_start,
                                double* fits_host, int* accepted_host, int* sweeps_done, double* fit_final,
                                void* stream);

/* Drop every cached als_sweep graph of this context and free the workspace
 * blocks it outgrew (a growing workspace keeps its old block, and the
 * graphs that use it, alive rather than wait for the device; they are
 * released here and by mtk_destroy).  Synchronises the device. */
mtk_status mtk_graph_reset(mtk_ctx* ctx);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of CP-ALS decompositions.
 *
 * A server owns a device, an HBM budget and a worker thread.  Requests
 * (a host FP32 tensor, rank R, sweep count) are admitted in arrival order
 * when a slot is free and their device block fits in the server's device
 * arena, whose footprint (device bytes actually allocated) never exceeds the
 * budget.  Every admitted request advances by one mode update per scheduler
 * step, and a step is one replay of a HIP graph captured when the server is
 * created: a grouped contraction over the tiles of all resident requests
 * (each at its own mode, shape and rank), a grouped inversion of their
 * normal-equation matrices, a grouped solve and a grouped normalisation,
 * driven by a device table with one entry per request.  Factor state stays
 * on the device until the request completes.  A request's result depends
 * only on its own inputs (its plan and summation orders are fixed by its
 * shape, rank, mode and precision), so it is bitwise the same alone and in
 * any mix.
 * --------------------------------------------------------------------- */
typedef struct mtk_server mtk_server;

typedef struct {
  int64_t id;              /* caller's request id */
  int32_t status;          /* mtk_status of the request */
  int32_t R;
  int64_t dims[3];
  double fit;              /* final fit (explicit residual) */
  double t_submit;         /* seconds since server start: submit call */
  double t_admit;          /* admitted to the device */
  double t_done;           /* result copied back to host */
} mtk_result;

/* budget_bytes: device bytes the server may hold for resident requests
 * (the arena grows in chunks of min(1 GiB, budget) and never past it).
 * max_slots: most requests resident at once (1 .. 64). */
mtk_status mtk_server_create(mtk_server** srv, int device, uint64_t budget_bytes,
                             int max_slots);

/* Submit one request.  x: HOST FP32 tensor (copied before return),
 * init: three HOST FP32 factor matrices (copied), prec: MTK_FP32 or
 * MTK_BF16X3.  factors_out (three host buffers dims[n] x R, may be NULL) and
 * lambda_out (host FP64[R], may be NULL) receive the result; they must stay
 * valid until the request is returned by mtk_server_poll.
 * Returns MTK_EBUDGET if the request can never fit the budget. */
mtk_status mtk_server_submit(mtk_server* srv, int64_t id, const float* x, const int64_t dims[3],
                             int64_t R, int prec, int sweeps, const float* const init[3],
                             float* const factors_out[3], double* lambda_out);

/* Device bytes a request of this shape, rank and precision (MTK_FP32 or
 * MTK_BF16X3) takes while resident: tensor, factors, lambda, partial sums,
 * solve and fit scratch.  0 for an invalid request.  Host-only. */
uint64_t mtk_server_request_bytes(const int64_t dims[3], int64_t R, int prec);

/* Retrieve up to `cap` finished requests (oldest first).  Waits up to
 * timeout_s seconds for at least one; returns the count in *n. */
mtk_status mtk_server_poll(mtk_server* srv, mtk_result* out, int cap, int* n, double timeout_s);

typedef struct {
  int32_t resident;             /* requests admitted and not yet returned */
  int32_t max_batch;            /* most requests carried by one step */
  uint64_t bytes_in_use;        /* device bytes of the resident requests' blocks */
  uint64_t peak_bytes_in_use;   /* largest bytes_in_use so far */
  uint64_t device_bytes;        /* device memory the arena holds (<= budget) */
  uint64_t steps;               /* scheduler steps launched */
} mtk_server_stat;

/* Counters of the server (a snapshot). */
mtk_status mtk_server_stats(mtk_server* srv, mtk_server_stat* out);

/* Finish every submitted request, then stop the worker and free the device
 * memory.  NULL is a no-op. */
mtk_status mtk_server_destroy(mtk_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MTTKRP_H_ */
