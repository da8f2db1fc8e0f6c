/*
 * libmlcc -- the contraction engine and diagnostics.
 *
 * Every Cholesky-index contraction of the method (Appendix A of Folkestad,
 * Kjonstad, Goletto, Koch, arXiv 2006.05226: the sums over J of products of
 * Cholesky vectors L^J_pq in the X1 basis, the Omega vectors and the Jacobian
 * transformations) runs on one batched, batch-reduced, strided GEMM.  This
 * header exposes that engine as a kernel-level entry point (unit tests,
 * tuning, callers that contract their own Cholesky blocks), a variant of it
 * that allocates nothing, a per-context tile override, per-contraction timing
 * and a read-out of internal intermediates for step-by-step parity tests.
 * Conventions (errors, contexts, streams) are those of mlcc.h.
 */
#ifndef MLCC_ENGINE_H
#define MLCC_ENGINE_H

#include "mlcc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- the engine ------------------------------------------------------------
 * Batched, batch-reduced strided GEMM on the device:
 *   C_z[m][n] = alpha * sum_{r<R} sum_{k<K} A_zr[m][k] B_zr[k][n] + beta * C_z[m][n]
 * with A_zr[m][k] at A + z*sA[3] + r*sA[2] + m*sA[0] + k*sA[1] and likewise
 * B (sB = {k, n, r, z}) and C (sC = {m, n, z}); strides in elements.  Device
 * pointers on the context's GPU only (MLCC_E_ARG otherwise).  prec:
 * MLCC_FP64 (A, B, C double; FP64 MFMA), MLCC_FP32 (A, B, C float; FP32 MFMA)
 * or MLCC_BF16X3 (A, B, C float; split BF16 products when A and B are both
 * contiguous along k and laid out for 16-byte loads, FP32 MFMA otherwise).
 * Reductions long enough to split are split over workgroups; the partial
 * sums go to a context workspace (allocated on first need, grown as needed,
 * charged to the context's budget) and are summed in a fixed order, so the
 * result is the same from run to run.  The call waits for its work. */
mlcc_status mlcc_gemm(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N, int64_t K,
                      int64_t R, int64_t Z, double alpha, const void *A, const int64_t sA[4],
                      const void *B, const int64_t sB[4], double beta, void *C,
                      const int64_t sC[3]);

/* As mlcc_gemm with two-level row and column indices: lvl = {Mlo, sA_m_hi,
 * sC_m_hi, Nlo, sB_n_hi, sC_n_hi}; row m has offset (m/Mlo)*hi + (m%Mlo)*lo
 * (lo = the ordinary stride), columns likewise; Mlo or Nlo 0 = one level. */
mlcc_status mlcc_gemm2(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N, int64_t K,
                       int64_t R, int64_t Z, double alpha, const void *A, const int64_t sA[4],
                       const void *B, const int64_t sB[4], double beta, void *C,
                       const int64_t sC[3], const int64_t lvl[6]);

/* ---- the plain-BF16 map of MLCC_BF16 -------------------------------------
 * tags: comma-separated contraction names (as mlcc_profile_get reports them)
 * whose products run as one BF16 product in MLCC_BF16 on this context, ""
 * for none, or NULL for the built-in map.  For tuning and for the accuracy
 * study that chose the built-in map.  Applies to problems and servers
 * created after the call; MLCC_E_ARG for a NULL context. */
mlcc_status mlcc_bf16_map(mlcc_context *ctx, const char *tags);

/* ---- the engine without allocation ----------------------------------------
 * For callers that cannot allocate device memory while they run: code being
 * captured into a HIP graph, tight serving loops, hosts that forbid
 * allocation after start-up.  The product of mlcc_gemm2 (lvl may be NULL for
 * one-level indices; same arguments and errors), except that:
 * - It allocates nothing: no hipMalloc / hipFree and no allocating library
 *   routine.  The partial sums of a split reduction go to a fixed device
 *   array of MLCC_NOALLOC_SCRATCH_BYTES that the library holds on every
 *   device it has created a context on, until the process ends; its address
 *   on each device is taken once, when the first context on that device is
 *   created.
 * - A product runs with at most as many reduction splits as that array holds
 *   (partial sums of M*N*Z elements of 8 bytes for MLCC_FP64, 4 otherwise,
 *   per split).  No size is refused for the array's sake: when two splits do
 *   not fit, the product runs unsplit.  Where it fits, the split count is the
 *   one mlcc_gemm2 uses, and the result is the same bit for bit; otherwise it
 *   differs only in the order of the partial sums.
 * - The work is enqueued on the context's stream and the call returns
 *   without waiting for it.
 * - Every call on one GPU uses that GPU's one array, which keeps the last
 *   call's contents.  Calls that overlap in time on one GPU (on different
 *   streams, contexts or host threads) race on it and give wrong results;
 *   calls ordered on one stream are safe.  No clearing is needed: a call
 *   writes every partial sum before it reads it.
 * MLCC_E_DEVICE if the array's address could not be taken on this device. */
#define MLCC_NOALLOC_SCRATCH_BYTES ((uint64_t)16 << 20)
mlcc_status mlcc_gemm_noalloc(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N, int64_t K,
                              int64_t R, int64_t Z, double alpha, const void *A,
                              const int64_t sA[4], const void *B, const int64_t sB[4],
                              double beta, void *C, const int64_t sC[3], const int64_t lvl[6]);

/* ---- tuning and diagnostics -------------------------------------------------
 * Tile override of the engine on this context, for parity tests and tuning:
 * later engine calls on the context's own stream (mlcc_gemm*, and the
 * problems of this context) whose tile menu lists the bm x bn output tile use
 * it, with the split count the cost model gives it; bm = bn = 0 restores the
 * cost model.  Server lanes are not affected.  last (may be NULL) receives
 * the tile of the context's previous engine call.  MLCC_E_ARG for a NULL
 * context or negative sizes. */
mlcc_status mlcc_gemm_tile(mlcc_context *ctx, int32_t bm, int32_t bn, int32_t last[2]);

/* Packed BF16 planes on this context, for parity tests and tuning.  Large
 * split- and plain-BF16 products first convert both operands into BF16
 * planes (hi, and lo for split products; rows padded to 256, the flattened
 * reduction index to 64) in an engine buffer of at most 3 GiB, then run a
 * kernel that streams the planes into LDS with direct loads.  mode 0: where
 * a cost rule says the conversion pays (the default), 1: wherever the product
 * allows it (no caller workspace, planes within the cap), -1: never.  The
 * products are the same BF16 products either way (same rounding, same
 * accumulation order within a k-step); results differ from the unpacked
 * kernel's only by the order of the FP32 sums across k-steps and splits.
 * Server lanes are not affected.  MLCC_E_ARG for a NULL context or a mode
 * outside -1..1. */
mlcc_status mlcc_gemm_planes(mlcc_context *ctx, int32_t mode);

/* Occupied indices per pair block of the MLCC2 doubles (the ground state
 * with the analytic s2 and the effective transformation build g~ and c2 per
 * occupied-pair block (I, J), I <= J) on problems of this context: occ > 0
 * forces blocks of occ occupied indices (the last one ragged), 0 restores the
 * memory rule (the largest blocks whose buffers fit in 4 GB).  For tests that
 * cover diagonal, off-diagonal and ragged blocks, and for tuning.  MLCC_E_ARG
 * for a NULL context or a negative occ. */
mlcc_status mlcc_pair_block_occ(mlcc_context *ctx, int32_t occ);

/* Per-contraction timing: when enabled, every GEMM-engine launch on the
 * context's stream is bracketed by HIP events and accumulated under the name
 * of the contraction it computes (e.g. "g_aibj", "ccs_vv").  flops counts
 * the algorithmic 2*M*N*K*R*Z of each launch.  Enabling clears the record. */
typedef struct {
  char name[40];
  int64_t launches;
  double ms;      /* summed kernel time of the GEMM launches */
  double flops;   /* summed algorithmic flops */
} mlcc_kernel_stat;
mlcc_status mlcc_profile_enable(mlcc_context *ctx, int32_t on);
/* Fills up to max entries, returns how many there are (synchronises). */
int32_t mlcc_profile_get(mlcc_context *ctx, mlcc_kernel_stat *out, int32_t max);

/* Internal intermediates for step-by-step parity tests.  which: 0 = F~ [n][n],
 * 1 = L~ [n_chol][n][n] (FP64 copy), 2 = g~_aibj [M][M] (only where the
 * problem stores it; MLCC_E_STATE otherwise), 3 = t1 [n_vir][n_occ], 4 =
 * doubles [M][M].  out is host memory of the stated size.  The values are
 * those of the last mlcc_residual / transform call. */
mlcc_status mlcc_debug_get(mlcc_problem *prob, int32_t which, double *out);

#ifdef __cplusplus
}
#endif

#endif /* MLCC_ENGINE_H */
