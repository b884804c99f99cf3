/*
 * mlh.h -- C ABI of the MI355X multilayer quasi-periodic Helmholtz solver.
 *
 * The library implements the robust periodizing integral-equation scheme of
 * Cho & Barnett, "Robust fast direct integral equation solver for
 * quasi-periodic scattering problems with a large number of layers"
 * (arXiv:1410.5003), for one GPU (gfx950):
 *
 *   - per-layer dense complex float64 fills of the Nystrom, proxy, wall and
 *     Rayleigh-Bloch blocks (Sec. 2, eq. (37), (38), (42)-(45), (56)-(63));
 *   - per-layer least-squares Schur eliminations of the proxy and Bragg
 *     unknowns (Sec. 3.1-3.2, eq. (67)-(78));
 *   - the block-tridiagonal LU sweep across layers (Sec. 3.3);
 *   - the multi-angle sweep with alpha-independent fill pieces (Sec. 3.4).
 *
 * Problem statement (Sec. 1): I periodic interfaces Gamma_1..Gamma_I (top to
 * bottom) with period d separate I+1 layers of real wavenumber k_1..k_{I+1};
 * a plane wave exp(i k_1 (cos t x + sin t y)), -pi < t < 0, is incident in the
 * top layer.  The outputs are the Bragg amplitudes a^U_n (reflected, top) and
 * a^D_n (transmitted, bottom) of the outgoing Rayleigh-Bloch expansions
 * eq. (7)-(8), their physical order labels n, and the flux-conservation error
 * eq. (86).
 *
 * Conventions
 *   - Unit cell -d/2 <= x < d/2.  All complex arrays are interleaved
 *     (re, im) float64 pairs.
 *   - Status codes only; no C++ exception crosses this interface.  After a
 *     failing call mlh_last_error() returns a message (thread-local).
 *   - The caller owns every input array; mlh_stack_create copies what it
 *     needs and keeps no caller pointer.  Outputs are caller-allocated.
 *   - All device work is enqueued on the context's HIP stream.  Calls with
 *     host outputs return after that work has finished.
 *   - Distinct handles may be used from distinct threads; one handle must
 *     not be used concurrently.
 */
#ifndef MLH_H
#define MLH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLH_ABI_VERSION 1

typedef int32_t mlh_status;
enum {
  MLH_OK = 0,
  MLH_E_INVALID_ARG = 1, /* bad size, pointer, angle or wavenumber          */
  MLH_E_GEOMETRY = 2,    /* interfaces cross, radiation lines or proxy
                            circles do not clear the layers                  */
  MLH_E_NOMEM = 3,       /* device allocation failed                         */
  MLH_E_DEVICE = 4,      /* a HIP call failed                                */
  MLH_E_SINGULAR = 5,    /* exact zero pivot in the block LU                 */
  MLH_E_UNSUPPORTED = 7  /* sizes beyond this library's limits              */
};

typedef struct mlh_ctx_s* mlh_ctx;
typedef struct mlh_stack_s* mlh_stack;

enum { MLH_IFACE_FOURIER = 0, MLH_IFACE_POLYGON = 1 };

/* One interface (Sec. 1; quadrature in Sec. 2.5, eq. (62)).
 * FOURIER: the graph y = y0 + sum_{m=1..n_modes} cos_coef[m-1] cos(2 pi m x/d)
 *          + sin_coef[m-1] sin(2 pi m x/d), discretised by the periodic
 *          trapezoid rule with n_nodes nodes s_j = 2 pi (j - 1/2)/n_nodes.
 * POLYGON: the periodic broken line through (vx[c], vy[c]), c = 0..n_vert-1,
 *          vx[0] = -d/2, vx[n_vert-1] = d/2, vy[0] = vy[n_vert-1], vx
 *          strictly increasing (a graph); vy and y0 are absolute heights, y0
 *          being the nominal height that places the proxy circles.  Segment c
 *          carries seg_nodes[c] >= 37 nodes of the Kress-graded trapezoid rule
 *          s_j = 2 pi (j - 1/2)/n on Z(w(s)) with grading exponent q >= 2
 *          (Sec. 2.5).  The singular self interaction is corrected per segment
 *          (Alpert's rule, periodic in s, no Bloch phase); segments interact
 *          through plain Nystrom entries.  A grading so strong that two nodes
 *          coincide in float64 is rejected (MLH_E_INVALID_ARG).
 * Both kinds: at most 512 nodes per interface (MLH_E_UNSUPPORTED beyond). */
typedef struct {
  int32_t kind;
  double y0;
  int32_t n_modes;
  const double* cos_coef;
  const double* sin_coef;
  int32_t n_nodes;
  int32_t n_vert;
  const double* vx;
  const double* vy;
  const int32_t* seg_nodes;
  double q;
} mlh_interface;

/* A stack (Sec. 1-2).  iface: I entries, top to bottom.  k: I+1 positive
 * wavenumbers, top layer first.  y_U > max Gamma_1 and y_D < min Gamma_I are
 * the radiation lines U and D.  P proxies per layer on a circle of radius R
 * about the layer centre (eq. (15)); M_w Gauss-Legendre wall nodes per layer
 * (eq. (61)); M_ud trapezoid nodes on U and on D; 2K+1 Rayleigh-Bloch orders
 * per side, the orders with kappa_n nearest 0 (M_ud >= 2K+1).  ls_mu is the
 * relative Tikhonov weight mu/||Q||_F of the least-squares Schur solves
 * (0 selects 1e-14). */
typedef struct {
  int32_t abi_version;
  int32_t I;
  const mlh_interface* iface;
  const double* k;
  double d, y_U, y_D;
  int32_t P;
  double R;
  int32_t M_w, M_ud, K;
  double ls_mu;
} mlh_stack_desc;

/* Bind a context to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
mlh_status mlh_ctx_create(int32_t device, void* hip_stream, mlh_ctx* out);
mlh_status mlh_ctx_destroy(mlh_ctx ctx);

/* Validate the description, build the quadrature geometry on the host,
 * allocate the stack's device memory and compute every alpha-independent
 * fill piece (the precomputation of Sec. 3.4).  Errors: MLH_E_INVALID_ARG,
 * MLH_E_GEOMETRY, MLH_E_UNSUPPORTED (checked before any device work),
 * MLH_E_NOMEM, MLH_E_DEVICE. */
mlh_status mlh_stack_create(mlh_ctx ctx, const mlh_stack_desc* desc, mlh_stack* out);

/* Recompute the alpha-independent fill pieces on the device (the same work
 * mlh_stack_create launches), e.g. to time the fill phase. */
mlh_status mlh_stack_refill(mlh_stack s);

mlh_status mlh_stack_destroy(mlh_stack s);

/* Sizes: n_den = 2 sum N_i density unknowns (eq. (64)); n_tot =
 * n_den + (I+1) P + 2 (2K+1) total unknowns (Sec. 3); device_bytes held. */
mlh_status mlh_stack_info(mlh_stack s, int64_t* n_den, int64_t* n_tot, int64_t* device_bytes);

/* Solve for n_angles incident angles theta[0..n_angles-1] (host array, each
 * in (-pi, 0)).  Angles are processed in batches that share the per-layer
 * kernels.  Outputs (host arrays, caller-allocated):
 *   aU, aD     [n_angles][2K+1] complex (interleaved), orders ascending;
 *   orders     [n_angles][2K+1] physical order labels n (may be NULL);
 *   flux_err   [n_angles] relative flux error eq. (86) with the incident
 *              vertical flux k_1 |sin theta| (may be NULL).
 * Errors: MLH_E_INVALID_ARG, MLH_E_SINGULAR, MLH_E_NOMEM, MLH_E_DEVICE. */
mlh_status mlh_solve(mlh_stack s, int32_t n_angles, const double* theta, double* aU,
                     double* aD, int32_t* orders, double* flux_err);

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

/* Per-kernel device times of one full step (refill + one-angle solve),
 * measured with HIP events on the context's stream around every launch. */
typedef struct {
  double fill_self_ms, fill_alpert_ms, fill_pairs_ms;
  double assemble_ms, rb_setup_ms, ls_panel_ms, ls_update_ms, ls_rhs_ms, schur_ms;
  double sweep_gemm_ms, gje_panel_ms, gje_update_ms, gje_rhs_ms, backsub_ms, bragg_ms;
  int32_t n_sweep_gemm, n_gje_panel, n_gje_update;
  double total_ms;
} mlh_profile;

/* Run one step (mlh_stack_refill + mlh_solve of angle theta) with HIP events
 * around each kernel launch and return the per-kernel times. */
mlh_status mlh_profile_step(mlh_stack s, double theta, mlh_profile* out);

/* The same for mlh_stack_refill + mlh_solve of n_angles angles (theta: host
 * array); times are summed over the batches the solve runs in.  The
 * instrumented run is not graph-captured. */
mlh_status mlh_profile_solve(mlh_stack s, int32_t n_angles, const double* theta, mlh_profile* out);

/* Launch choices of the solve (the dense factorisations of Sec. 3.2-3.3
 * and the batched sweep of Sec. 3.4).  None changes what is computed; the
 * placement of the right-hand sides changes the rounding order only.
 *   rhs_in_step_pct  a cyclic-reduction level eliminates its right-hand
 *                    sides inside the Gauss-Jordan steps (no replay after
 *                    the last step) when its widest step launch needs at
 *                    most rhs_in_step_pct workgroups per 100 compute units;
 *                    0 = never.  Range 0..1000.
 *   ls_row_blocks    16-row blocks per wavefront of the least-squares
 *                    right-hand-side kernels for layers of at most 384
 *                    rows: 3 or 4 (larger layers always take 4).
 *   gje_rhs_cols     columns per workgroup of the Gauss-Jordan replay for
 *                    orders up to 608: 16 or 8 (larger orders take 8).
 *   asm_in_panels    1: the block-system assembly runs inside the
 *                    least-squares panel launches, on the compute units
 *                    they leave idle; 0: in a launch of its own.
 * A new stack starts with {300, 3, 16, 1}. */
typedef struct {
  int32_t rhs_in_step_pct;
  int32_t ls_row_blocks;
  int32_t gje_rhs_cols;
  int32_t asm_in_panels;
} mlh_tuning;

/* Read or replace the stack's launch choices.  set: MLH_E_INVALID_ARG for a
 * value outside the ranges above (the stack keeps its choices). */
mlh_status mlh_stack_get_tuning(mlh_stack s, mlh_tuning* out);
mlh_status mlh_stack_set_tuning(mlh_stack s, const mlh_tuning* t);

/* Autotune: time mlh_solve of these n_angles angles (host array, as for
 * mlh_solve) under candidate launch choices, one field at a time with the
 * others at their best so far (every field's values above; rhs_in_step_pct
 * from {0, 100, 150, 200, 300, 500, 1000}), taking the fastest of `reps` timed
 * solves (reps >= 1) after one untimed solve per candidate; keep the
 * fastest choices in the stack and return them in out (may be NULL).
 * Errors: those of mlh_solve; the stack then keeps its previous choices. */
mlh_status mlh_stack_autotune(mlh_stack s, int32_t n_angles, const double* theta, int32_t reps,
                              mlh_tuning* out);

const char* mlh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLH_H */
