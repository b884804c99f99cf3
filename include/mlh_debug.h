/*
 * mlh_debug.h -- inspection calls of the MI355X multilayer quasi-periodic
 * Helmholtz solver (include/mlh.h): copies of intermediate device results for
 * the stage-by-stage parity tests.  They are not part of the solver's
 * problem-statement interface (Sec. 1 of Cho & Barnett, arXiv:1410.5003) and
 * synchronise the context's stream.
 */
#ifndef MLH_DEBUG_H
#define MLH_DEBUG_H

#include "mlh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Inspection (used by the parity tests): copy one alpha-independent fill
 * piece to host memory `out` (column-major, leading dimension = rows,
 * complex interleaved).  which: 0 A_self[i] (piece p = 0,1,2 for copies
 * l = -1,0,1), 1 A_up[i] (rows Gamma_i, cols Gamma_{i+1}), 2 A_dn[i] (rows
 * Gamma_{i+1}, cols Gamma_i), 3 B_own[i], 4 B_below[i], 5 C_own[j]
 * (p = 0: target x+2d, 1: x-d), 6 C_above[j], 7 Q[j] (p = 0: x+d, 1: x),
 * 8 Z_U (p = copy), 9 Z_D, 10 V_U, 11 V_D.  rows/cols receive the shape
 * (out may be NULL to query it). */
mlh_status mlh_debug_get_piece(mlh_stack s, int32_t which, int32_t index, int32_t piece,
                               double* out, int32_t* rows, int32_t* cols);

/* Inspection: evaluate the device Hankel routine at n host arguments x > 0:
 * out[4*i..4*i+3] = (Re, Im) of H0^(1)(x) and of g1m(x) = (i pi x/2) H1^(1)(x) - 1. */
mlh_status mlh_debug_hankel(mlh_ctx ctx, int32_t n, const double* x, double* out);

/* Inspection: complex batched GEMM C = C + alpha A B (column-major, host
 * arrays, m x k times k x n), run with the library's FP64-MFMA kernel. */
mlh_status mlh_debug_zgemm(mlh_ctx ctx, int32_t m, int32_t n, int32_t k, const double* alpha,
                           const double* A, const double* B, double* C);

/* Inspection: run the solve for one angle up to phase `stop_phase`
 * (1: blocks assembled for alpha, 2: + per-layer least squares, 3: + Schur
 * complements, 4: + sweep) and keep that angle's workspace for
 * mlh_debug_get_work. */
mlh_status mlh_debug_solve_partial(mlh_stack s, double theta, int32_t stop_phase);

/* Inspection: copy a workspace block of the last mlh_debug_solve_partial:
 * which 0 [A'_ii | f~_i] (n_i x (n_i+1)), 1 A'_{i,i+1}, 2 A'_{i+1,i},
 * 3 stacked least-squares matrix of layer j ((m+c) x c), 4 its right-hand
 * side / solution ((m+c) x ncol), 6 eta_i (densities, phase 4).  Column-major,
 * complex interleaved; out may be NULL to query the shape. */
mlh_status mlh_debug_get_work(mlh_stack s, int32_t which, int32_t index, double* out, int32_t* rows,
                              int32_t* cols);

#ifdef __cplusplus
}
#endif
#endif /* MLH_DEBUG_H */
