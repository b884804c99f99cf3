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

#define MLH_ABI_VERSION 2

typedef int32_t mlh_status;
enum {
  MLH_OK = 0,
  MLH_E_INVALID_ARG = 1, /* bad size, pointer, angle or wavenumber          */
  MLH_E_GEOMETRY = 2,    /* interfaces cross, radiation lines or proxy
                            circles do not clear the layers                  */
  MLH_E_NOMEM = 3,       /* device allocation failed                         */
  MLH_E_DEVICE = 4,      /* a HIP call failed                                */
  MLH_E_SINGULAR = 5,    /* exact zero pivot in the block LU                 */
  MLH_E_ACCURACY = 6,    /* flux error beyond the tolerance the caller set
                            (mlh_stack_set_flux_tolerance; outputs written)  */
  MLH_E_UNSUPPORTED = 7  /* sizes beyond this library's limits              */
};

typedef struct mlh_ctx_s* mlh_ctx;
typedef struct mlh_stack_s* mlh_stack;
typedef struct mlh_batch_s* mlh_batch;

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
 * in (-pi, 0)): the Schur eliminations of Sec. 3.2, the block-tridiagonal
 * solve of Sec. 3.3 for the densities eta, and the Bragg amplitudes
 * x_1 = -X_1 eta_1, x_{I+1} = -X_{I+1} eta_I with the flux error eq. (86).
 * Angles whose Bloch phases alpha agree share one factorisation (Sec. 3.4);
 * batches of systems share the per-layer launches.  A batch holds as many
 * systems as 80 % of the free device memory takes, or, when the environment
 * variable MLH_WORKSPACE_LIMIT_MB is a positive number, as that many MiB
 * take (at least one system per batch); the stack keeps its workspace for
 * later calls.
 *
 * outputs_on_device: 0 = the output pointers are host memory and the call
 * returns once they are written; 1 = they are device memory of the
 * context's device (e.g. torch tensors) and the call returns once the work
 * and the output copies are enqueued on the context's stream (the caller
 * synchronises that stream before reading them; an exact zero pivot is then
 * not reported).  Outputs, caller-allocated:
 *   aU, aD     [n_angles][2K+1] complex (interleaved), orders ascending;
 *   orders     [n_angles][2K+1] physical order labels n (may be NULL);
 *   flux_err   [n_angles] relative flux error eq. (86) with the incident
 *              vertical flux k_1 |sin theta| (may be NULL);
 *   eta        [n_angles][N_den] complex densities [tau_1; sigma_1; ...;
 *              tau_I; sigma_I] of eq. (64), interfaces top to bottom (may be
 *              NULL).  The densities are fixed only up to the least-squares
 *              choice of Sec. 3.2 (its closing Remark); the amplitudes are not.
 * Errors: MLH_E_INVALID_ARG, MLH_E_SINGULAR, MLH_E_ACCURACY (only after
 * mlh_stack_set_flux_tolerance; every output is still written), MLH_E_NOMEM,
 * MLH_E_DEVICE. */
mlh_status mlh_solve(mlh_stack s, int32_t n_angles, const double* theta, int32_t outputs_on_device,
                     double* aU, double* aD, int32_t* orders, double* flux_err, double* eta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mlh_solve
 * with the same arguments, outputs and errors, whose solve workspace lives
 * in a fixed per-device area of 64 MiB reserved when the library is loaded
 * on that device (held until the process ends) instead of memory the stack
 * allocates.  The call allocates nothing on the device, captures no graph and
 * launches its kernels on the context's stream one by one.  The stack's own
 * fill pieces stay where mlh_stack_create put them.  Angles are solved in as
 * many passes as the area needs; a stack one of whose systems (one Bloch
 * phase and its angles) needs more than 64 MiB of workspace is rejected with
 * MLH_E_UNSUPPORTED before any device work.  Every call on one device uses
 * the same area: calls that overlap in time on one device (two host threads,
 * or two streams) race and must be serialised by the caller. */
mlh_status mlh_solve_noalloc(mlh_stack s, int32_t n_angles, const double* theta, int32_t outputs_on_device,
                             double* aU, double* aD, int32_t* orders, double* flux_err, double* eta);

/* Opt in to an accuracy report: with tol > 0, mlh_solve returns
 * MLH_E_ACCURACY when some angle's |flux error| (eq. (86)) exceeds tol; with
 * device outputs it then waits for the stream to read the flux errors.
 * tol = 0 (the default) turns the check off.  Errors: MLH_E_INVALID_ARG for a
 * negative or non-finite tol. */
mlh_status mlh_stack_set_flux_tolerance(mlh_stack s, double tol);

/* Per-kernel device times of one full step (refill + solve), measured with
 * HIP events on the context's stream around every launch.  The launches are
 * those of the captured graph, run one at a time on one stream: the fused
 * Gauss-Jordan step kernel where the graph uses it (gje_step_ms), the panel
 * and update kernels where the graph runs them on two streams.
 *   *_ms         summed device time of the group's launches;
 *   n_*          its launch count;
 *   *_flops      the real float64 flops of the group's complex products,
 *                8 m n k per product of an m x k by a k x n matrix (the
 *                descriptors' own sizes; the three-real-product evaluation
 *                is not what is counted). */
typedef struct {
  double fill_self_ms, fill_alpert_ms, fill_pairs_ms;
  double assemble_ms, rb_setup_ms, ls_panel_ms, ls_update_ms, ls_rhs_ms, schur_ms;
  double sweep_gemm_ms, gje_panel_ms, gje_update_ms, gje_rhs_ms, backsub_ms, bragg_ms;
  int32_t n_sweep_gemm, n_gje_panel, n_gje_update;
  double total_ms;
  double gje_step_ms;
  int32_t n_gje_step, n_schur_gemm, n_gje_rhs, n_backsub;
  double schur_flops, sweep_gemm_flops;
  /* Gauss-Jordan work counted as LU with partial pivoting plus triangular
   * solves, (8/3) n^3 + 8 n^2 r for an order-n block with r right-hand-side
   * columns: gje_step_flops for the levels run by the step kernel (their
   * right-hand sides included when eliminated inside the steps),
   * gje_panel_update_flops for the levels run by the panel and update
   * kernels, gje_rhs_flops for right-hand sides replayed afterwards. */
  double gje_step_flops, gje_panel_update_flops, gje_rhs_flops;
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
 *   gje_rhs_cols     columns per workgroup of the Gauss-Jordan replay: 16
 *                    (an LDS tile up to order 608, a register tile above)
 *                    or 8 (LDS tiles: 8 columns, 10 for orders 609-1008).
 *   asm_in_panels    1: the block-system assembly runs inside the
 *                    least-squares panel launches, on the compute units
 *                    they leave idle; 0: in a launch of its own.
 *   gemm_slab_k      depth of the K slabs of the complex GEMMs (Schur
 *                    updates and cyclic-reduction products), staged in two
 *                    LDS buffers: 8 (32 KiB a workgroup) or 16 (64 KiB).
 * A new stack starts with {300, 3, 16, 1, 8}. */
typedef struct {
  int32_t rhs_in_step_pct;
  int32_t ls_row_blocks;
  int32_t gje_rhs_cols;
  int32_t asm_in_panels;
  int32_t gemm_slab_k;
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

/* Launch-choice cache.  Every successful autotune (stack or batch) records
 * the choices it kept under a key made of the device's architecture name
 * (hipDeviceProp_t::gcnArchName) and the size class of the work: interface
 * count (power-of-two bucket), block orders (all up to 576, up to 608, above,
 * or mixed), least-squares rows (all up to 384, above, or mixed) and the
 * number of systems solved at once (distinct Bloch phases among the angles,
 * or the batch's stacks; buckets 1, 2-4, 5-16, 17-64, more).  The cache
 * lives for the process; when the environment variable MLH_TUNING_CACHE
 * names a file, each record is also appended to it and the file is read
 * (later lines win, invalid ones are skipped) before the first lookup.
 * mlh_stack_tune_cached: if a record exists for this stack and these angles
 * (host array, each in (-pi, 0)), the stack takes it and *found = 1;
 * otherwise *found = 0 and the stack keeps its choices.  out (may be NULL)
 * receives the stack's choices either way.  MLH_E_INVALID_ARG for NULL
 * s/theta/found, n_angles < 1 or an angle out of range. */
mlh_status mlh_stack_tune_cached(mlh_stack s, int32_t n_angles, const double* theta, mlh_tuning* out,
                                 int32_t* found);

/* Field evaluation (Sec. 3.3, last paragraph): solve the stack for incident
 * angle theta, then evaluate the scattered field u at n_pts targets
 * (x[t], y[t]) (host arrays; n_pts >= 0).  A target inside layer j takes
 * that layer's representation eq. (16)-(18): the near-field single- and
 * double-layer potentials of the interfaces bounding it, each over the
 * copies l = -1, 0, 1 with phase alpha^l (eq. (14)), plus the layer's proxy
 * expansion with the strengths of the least-squares solve (eq. (15)).  A
 * target with y >= y_U takes the Rayleigh-Bloch expansion eq. (7) with the
 * computed a^U, one with y <= y_D eq. (8) with a^D.  Targets outside the unit
 * cell are mapped into it by quasi-periodicity (eq. (6)).  The incident wave
 * eq. (1) is not included: the total field is u plus the incident wave in
 * layer 1 and above U.  The potentials use the plain quadrature of the
 * off-diagonal Nystrom entries: spectrally accurate a few node spacings
 * away from the interfaces, not corrected closer to them.
 * Outputs: u [n_pts] complex (interleaved); layer [n_pts] region of each
 * target, -1 above U, 0..I the layers top to bottom, I+1 below D (may be
 * NULL); host or device memory per outputs_on_device (the call returns
 * once they are written either way).  The stack's solve workspace then
 * holds this angle's solution.  Errors: MLH_E_INVALID_ARG (also for a
 * non-finite target), MLH_E_NOMEM, MLH_E_DEVICE, those of mlh_solve. */
mlh_status mlh_field(mlh_stack s, double theta, int64_t n_pts, const double* x, const double* y,
                     int32_t outputs_on_device, double* u, int32_t* layer);

/* Gradient of J = sum_a e^U_0(theta[a]), the zeroth-order reflected
 * efficiencies (eq. (86); e^U_0 = |a^U_0|^2 since k^U_0 = k_1 |sin theta|),
 * by the adjoint of the solve (Sec. 3.2-3.3 transposed): the forward solve;
 * the transposed block-tridiagonal solve A'^T z = w with w the row of X_1
 * that yields a^U_0; the least-squares adjoint vectors l_j = (Q'_j^+)^T v_j
 * from the layers' QR factors; then the derivative of every block contracted
 * with the adjoint and forward vectors, da0 = -l^T dE u (the fills are
 * recomputed, not stored):
 *   grad_k[I+1]  dJ/dk_j from the wavenumber derivatives of every
 *                alpha-independent piece (dS/dk = -g1/(2 pi k), dD/dk =
 *                n'.dv (i/4) k H0, ...; the self blocks with the Alpert
 *                correction applied to the derivative kernels).  The incident
 *                medium's k_1 also sets the Bloch phase and the Rayleigh-Bloch
 *                orders; its derivative is not formed: grad_k[0] = NaN;
 *   grad_shape   (may be NULL) dJ/d(cos_coef), dJ/d(sin_coef) of every
 *                FOURIER interface, interface by interface, n_modes cos
 *                entries then n_modes sin entries (POLYGON interfaces take no
 *                entries): the pieces of the blocks that touch the interface
 *                (its self block, the neighbour pairs, the proxy rows, the
 *                wall columns, the U/D rows and the incident right-hand side
 *                on interface 1) differentiated by central differences of
 *                the fill kernels at perturbed node geometry (step 1e-5 of the
 *                largest coefficient); the wall nodes, whose end points follow
 *                the interface heights at x = -d/2, are held fixed.
 * theta: n_angles host angles in (-pi, 0), all in one batch of systems.
 * The device scratch the call needs (about the size of the stack's
 * alpha-free pieces, plus a few GB for the shape passes) stays with the
 * stack for later calls until mlh_stack_destroy; a call that needs more
 * replaces it.
 * Outputs (host): J_out (may be NULL), grad_k, grad_shape.  Errors:
 * MLH_E_INVALID_ARG (also when the zeroth order leaves the window),
 * MLH_E_UNSUPPORTED (too many angles for one batch), MLH_E_NOMEM,
 * MLH_E_DEVICE. */
mlh_status mlh_adjoint(mlh_stack s, int32_t n_angles, const double* theta, double* J_out, double* grad_k,
                       double* grad_shape);

/* Batches of independent stacks (many unrelated structures at once; the
 * per-layer independence of the Schur eliminations, Sec. 3.2, and of the
 * block eliminations, Sec. 3.3, holds across stacks too).  A batch solves
 * one incident angle per stack with the work of all its stacks sharing
 * every launch: the fill launches (with refill), the least-squares, Schur
 * and assembly launches, and level l of every stack's block-tridiagonal
 * reduction in the launches of level l.  The launch sequence is captured in
 * a HIP graph and replayed while the batch and its launch choices stay the
 * same.
 *
 * mlh_batch_create: the stacks (n_stacks >= 1, distinct, created on the
 * context's device) stay owned by the caller and must outlive the batch;
 * the batch holds their merged fill job tables.  Errors: MLH_E_INVALID_ARG,
 * MLH_E_NOMEM, MLH_E_DEVICE. */
mlh_status mlh_batch_create(mlh_ctx ctx, int32_t n_stacks, const mlh_stack* stacks, mlh_batch* out);
mlh_status mlh_batch_destroy(mlh_batch b);

/* Solve stack s of the batch for incident angle theta[s] (host array of
 * n_stacks angles, each in (-pi, 0)).  refill = 1 first recomputes every
 * stack's alpha-independent fill pieces (mlh_stack_refill of all of them,
 * in three launches); 0 uses the pieces in place.  outputs_on_device as for
 * mlh_solve.  Outputs, caller-allocated, stacks in batch order:
 *   aU, aD    the 2K_s+1 Bragg amplitudes of each stack, concatenated
 *             (sum_s (2K_s+1) complex, interleaved);
 *   orders    their order labels, concatenated (may be NULL);
 *   flux_err  [n_stacks] flux errors eq. (86) (may be NULL);
 *   stack_ms  [n_stacks] host array (may be NULL): device clock time from
 *             the first launch of the solve to the write of each stack's
 *             results, in ms (the call then waits for the stream).
 * Errors: those of mlh_solve (no accuracy report). */
mlh_status mlh_batch_solve(mlh_batch b, const double* theta, int32_t refill, int32_t outputs_on_device, double* aU,
                           double* aD, int32_t* orders, double* flux_err, double* stack_ms);

/* Launch choices of a batch (the fields of mlh_tuning; a new batch starts
 * with {300, 3, 16, 1, 8}), and their autotune: mlh_stack_autotune's search,
 * timing whole mlh_batch_solve calls (no refill) of the angles theta[s]. */
mlh_status mlh_batch_get_tuning(mlh_batch b, mlh_tuning* out);
mlh_status mlh_batch_set_tuning(mlh_batch b, const mlh_tuning* t);
mlh_status mlh_batch_autotune(mlh_batch b, const double* theta, int32_t reps, mlh_tuning* out);
/* The cache lookup of mlh_stack_tune_cached for a batch (its size class:
 * all its stacks' interfaces, block orders and layers, one system per
 * stack). */
mlh_status mlh_batch_tune_cached(mlh_batch b, mlh_tuning* out, int32_t* found);

const char* mlh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLH_H */
