// Internal declarations shared by the host orchestration and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "hankel.hpp"

namespace mlh {

// ---------------------------------------------------------------------------
// fill jobs: one (target set) x (source set) block, up to three shifted pieces
// ---------------------------------------------------------------------------
// kFillPair: the layer potentials between two curves in both directions at
// once (targets on the first as the job's out, targets on the second as
// out_t), one Hankel evaluation per pair and copy
enum FillKind : int { kFillLayerPotential = 0, kFillProxy = 1, kFillPair = 2 };

struct FillJob {
  const double* tx;
  const double* ty;
  const double* tnx;   // null: constant normal (cnx, cny)
  const double* tny;
  const double* sx;
  const double* sy;
  const double* snx;
  const double* sny;
  const double* sw;    // source weights (layer potentials only)
  double cnx, cny;
  double dy0;          // (target base height) - (source base height)
  double k;
  double scale;
  double tshift[3];
  double sshift[3];
  cplx* out[3];
  int Mt, Ns, ld, kind, npieces;
  int tile_begin, tiles_m;  // kFillPair: 16 x 16 tiles, else kFillTileM x kFillTileN
  // kFillPair only: the reverse block (targets = sources above), its pieces
  // in reverse copy order, leading dimension, weights (of the targets above)
  // and sign
  cplx* out_t[3];
  int ld_t;
  const double* tw;
  double scale_t;
  int dk;  // 1: write the wavenumber derivative dK/dk of every entry instead (no jump terms)
};

// largest grid of one launch (workgroups); bigger launches are split
constexpr int kMaxLaunchBlocks = 1 << 22;

constexpr int kFillTileM = 64;
constexpr int kFillTileN = 4;
constexpr int kSelfTile = 16;  // self blocks: 16 x 16 blocks of the upper triangle

// self block of one interface: difference kernels at ka (above) and kb (below)
struct SelfJob {
  const double* x;
  const double* y;
  const double* nx;
  const double* ny;
  const double* w;
  const int* seg_lo;   // cornered interface: first node of each node's segment
  const int* seg_len;  //   and that segment's node count (null: smooth)
  double ka, kb, d;
  cplx* out[3];   // pieces l = -1, 0, 1 (n x n, ld = n)
  int N;
  int tile_begin, tiles_m;  // tiles_m: 16-node blocks per side (upper-triangle tiles)
  int dk;         // 0: the block; 1: its derivative in ka; 2: in kb (no jump terms)
};

// Alpert correction of one interface: aux invariants per (target, aux)
struct AlpertJob {
  const double* r2;
  const double* nd;
  const double* npd;
  const double* nn;
  const double* cw;   // smooth: aux weight u_k h |Z'|; cornered: u_k
  const double* t;    // aux position in node-index units (segment-local if cornered)
  const int* seg_lo;  // cornered interface: segment of each node (null: smooth)
  const int* seg_len;
  const double* colw; // cornered interface: node weights w_j (interpolation of density x Jacobian)
  double ka, kb;
  cplx* out[3];
  int N;
  int block_begin;
  int dk;         // as SelfJob::dk
};

constexpr int kAlpertAux = 30;     // 2 x 15 auxiliary nodes per target
constexpr int kAlpertStencil = 16; // Lagrange interpolation stencil

// ---------------------------------------------------------------------------
// alpha assembly: dst = sum_p coef[p] * src[p] elementwise (up to 3 pieces),
// rows x cols sub-block with its own leading dimensions
// ---------------------------------------------------------------------------
struct AsmJob {
  const cplx* src[3];
  cplx* dst;
  cplx coef[3];
  int npieces;
  int rows, cols, lds, ldd;
  int tile_begin;  // first kAsmTile-element tile of this job in the launch
};
constexpr int kAsmTile = 2048;  // elements per assembly workgroup (8 per thread)

// batched complex GEMM  C += alpha (A B + A2 B2)  (column-major); the second
// product (k2 may be 0) lets one descriptor own its output tile, so no two
// workgroups of a launch ever update the same C entry
constexpr int kGemmTile = 64;  // output tile of one zgemm workgroup (kGemmTile x kGemmTile)

struct GemmDesc {
  const cplx* A;
  const cplx* B;
  const cplx* A2;
  const cplx* B2;
  const cplx* C0;  // C = C0 + alpha (...); C0 = C updates in place, null starts from zero
  cplx* C;
  cplx alpha;
  int m, n, k, lda, ldb, k2, lda2, ldb2, ldc, ldc0;
  int tile_begin, tiles_m;
};




// host-side launchers (kernels_*.hip)
// dk: the wavenumber-derivative pieces of jobs whose dk field is set
void launch_fill(const FillJob* d_jobs, int njobs, int total_tiles, hipStream_t st, bool dk = false);
void launch_self(const SelfJob* d_jobs, int njobs, int total_tiles, int a_excl, hipStream_t st, bool dk = false);
void launch_alpert(const AlpertJob* d_jobs, int njobs, int total_blocks, int a_excl, hipStream_t st,
                   bool dk = false);
void launch_assemble(const AsmJob* d_jobs, int njobs, int total_tiles, hipStream_t st);
void launch_gemm(const GemmDesc* d_desc, int ndesc, int total_tiles, hipStream_t st, int slab_k = 8);
void launch_hankel_eval(const double* x, double* out, int n, hipStream_t st);

}  // namespace mlh

namespace mlh {

// constants of the stack an angle belongs to
struct StackConsts {
  const double* x1;     // Gamma_1 nodes (x, y relative to y0_1, normals)
  const double* y1;
  const double* nx1;
  const double* ny1;
  const double* xud;    // U / D node abscissae
  double y0_1;
  double d, k1, kI1;
  int N1, NI, Mw, Mud, P, K;
};

// per-angle radiation rows, right-hand side and Bragg/flux extraction
struct AngleDesc {
  StackConsts sc;
  double theta;
  int owner;      // first angle of its system: writes the shared W rows
  cplx* S0;       // layer-1 stacked LS matrix (W_U goes at rows 2 M_w.., cols P..)
  cplx* SI;       // layer-(I+1) stacked LS matrix (W_D)
  int ldS0, ldSI;
  cplx* F0;       // right-hand side of interface 1 (n_1 entries)
  const cplx* X0; // layer-1 least-squares solution, ld ldX0 (rows P.. are a^U rows)
  const cplx* XI; // layer-(I+1) least-squares solution
  int ldX0, ldXI;
  const cplx* eta0;
  const cplx* etaI;
  cplx* aU;
  cplx* aD;
  int* orders;
  double* flux;
  unsigned long long* tdone;  // null, or: device clock when the angle's results are written
};



void launch_rb_setup(const AngleDesc* d_ang, int nang, hipStream_t st);
// device clock (wall_clock64) into *p
void launch_stamp(unsigned long long* p, hipStream_t st);
void launch_bragg(const AngleDesc* d_ang, int nang, hipStream_t st);

// densities eta of a batch gathered into one row of N_den entries per angle
struct EtaSeg {      // per interface of each system of a batch
  int64_t src_off;   // byte offset of eta_i in the system's workspace
  int64_t dst_off;   // offset of interface i within an angle's row
  int n;             // n_i
};
struct EtaDst {      // per angle
  const char* sys_base;  // its system's workspace
  int col;               // its column in the system's eta blocks
  int seg0, nseg;        // its system's segments
  cplx* dst;             // its output row (N_den entries)
};
// grid: max_seg segments (of at most max_n entries) per angle
void launch_gather_eta(const EtaSeg* d_seg, int max_seg, int max_n, const EtaDst* d_dst, int ndst, hipStream_t st);

// ---------------------------------------------------------------------------
// field evaluation (kernels_field.hip)
// ---------------------------------------------------------------------------
// c = -X[0:P, 0:n0] eta0 - X[0:P, n0:n0+n1] eta1 for one layer
struct ProxyStrengthJob {
  const cplx* X;  // least-squares solution, ld ldX
  const cplx* eta0;
  const cplx* eta1;
  cplx* c;        // P proxy strengths
  int ldX, n0, n1, P;
};
struct FieldCurve {  // one bounding interface of a layer (N = 0: none)
  const double* x;
  const double* y;   // relative to y0
  const double* nx;
  const double* ny;
  const double* w;
  const cplx* eta;   // [tau; sigma], 2N entries
  double y0;
  int N;
};
struct FieldRegion {
  int kind;          // 0: a layer; 1: above U; 2: below D
  int label;         // -1 above U, 0..I the layers, I+1 below D
  double k;          // the region's wavenumber
  FieldCurve above, below;
  const double* px;  // proxies (y relative to centre)
  const double* py;
  const double* pnx;
  const double* pny;
  double centre;
  const cplx* coef;  // proxy strengths of the layer
  const cplx* amp;   // kind 1 / 2: Bragg amplitudes a^U / a^D
  double yline;      // kind 1 / 2: y_U / y_D
};
struct FieldTarget {  // a target mapped into the unit cell
  double x, y;
  double ph_re, ph_im;  // alpha^m of its cell
  int64_t idx;          // position in the caller's arrays
};
struct FieldTile {
  int region, first, count;
};
struct FieldConsts {
  cplx alpha_pow[3];  // alpha^{-1}, 1, alpha
  double d, kappa0;
  int n0, K, nK, P;
};
void launch_proxy_strength(const ProxyStrengthJob* d_jobs, int njobs, hipStream_t st);
void launch_field(const FieldTile* d_tiles, int ntiles, const FieldRegion* d_regions, const FieldTarget* d_tgt,
                  double* u, int* layer_out, const FieldConsts& fc, hipStream_t st);

// ---------------------------------------------------------------------------
// adjoint (kernels_adjoint.hip)
// ---------------------------------------------------------------------------
struct TransposeJob {  // dst (rows x cols, ld ldd) = src^T (src cols x rows, ld lds); src null: zeros
  const cplx* src;
  cplx* dst;
  int lds, ldd, rows, cols;
  int tile_begin;      // first 32 x 32 tile of the job in the launch
};
struct BtzJob {        // v[0:c]: v[p] = sum_r B1[p ld1 + r] z1[r] + B2[..] z2[..] (p < P), + 1 at unit
  const cplx* B1;
  const cplx* z1;
  const cplx* B2;
  const cplx* z2;
  cplx* v;
  int ld1, n1, ld2, n2, P, c, unit;
};
struct LsAdjJob {      // ell[0:m] = (Q'^+)^T v from the QR [Q'; mu I] = Q_f R kept in S, T
  const cplx* S;       // M x c factored matrix (R above the diagonal, reflectors below)
  const cplx* T;       // per panel 16 x 16 block-reflector factor
  const cplx* v;
  cplx* ell;
  int M, m, c;
};
struct BilinJob {      // acc[out] += scale * left^T (sum_p coef_p P_p) right
  const cplx* P[6];
  cplx coef[6];
  const cplx* left;
  const cplx* right;
  double scale;
  int np, rows, cols, ld, out;
  int tile_begin;      // first 64 x 64 tile of the job in the launch
};
void launch_transpose(const TransposeJob* d, int njobs, int tiles, hipStream_t st);
void launch_btz(const BtzJob* d, int njobs, hipStream_t st);
void launch_ls_adjoint(const LsAdjJob* d, int njobs, hipStream_t st);
void launch_bilinear(const BilinJob* d, int njobs, int tiles, double* acc, hipStream_t st);

// Fixed workspace of the allocation-free solve: kScratchBytes per device,
// shared by every such call on that device (calls that overlap on one device
// race).  scratch_address returns the device's own copy; the device must be
// current.
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(int device, char** ptr);

}  // namespace mlh

namespace mlh {

// Blocked Gauss-Jordan solve with partial pivoting of W = [A | B] (n x ncol,
// column-major, ld = n): after all panels W[:, n:] = A^{-1} B.
// two incident angles share a system when their kappa_0 d/(2 pi) agree modulo
// 1 to this tolerance (alpha = exp(i kappa_0 d) then agrees to about 1e-11)
constexpr double kAlphaTol = 1e-12;

// Kernels reach device memory through pointers held in descriptors, whose
// address space the compiler cannot infer; these casts let it emit global
// rather than flat memory instructions.  Global accesses count against the
// vector-memory counter only, so a wait for LDS data does not also wait for
// every load still in flight.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
typedef double gdouble2 __attribute__((ext_vector_type(2)));
// one complex value from / to device memory, as a 16-byte global access
__device__ __forceinline__ double2 ldc(const cplx* p) {
  const gdouble2 v = *gmem(reinterpret_cast<const gdouble2*>(p));
  return make_double2(v.x, v.y);
}
// p's value when ok, zero otherwise.  p must be a valid address either way
// (callers clamp their indices), so no branch guards the load and loads
// issue back to back instead of one wait per guarded load.
__device__ __forceinline__ double2 ldc_sel(const cplx* p, bool ok) {
  const double2 v = ldc(p);
  return make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
}
__device__ __forceinline__ void stc(cplx* p, double re, double im) {
  gdouble2 v;
  v.x = re;
  v.y = im;
  *gmem(reinterpret_cast<gdouble2*>(p)) = v;
}

// Assembly of one kAsmTile-element tile by 256 threads: 8 elements per
// thread, consecutive threads on consecutive rows.  Every source load of a thread is issued
// before the first result is formed (clamped addresses, no branch), and the
// indices are 32-bit: a job holds at most a few million elements, since the
// block orders are bounded when the stack is validated.
template <int NP, int B>  // NP source pieces, B elements of a thread in flight at once
__device__ __forceinline__ void assemble_tile(const AsmJob& J, int base) {
  const int rows = J.rows, total = rows * J.cols, lds = J.lds, ldd = J.ldd;
#pragma unroll
  for (int g = 0; g < kAsmTile / 256; g += B) {
    uint32_t so[B], dofs[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = min(base + 256 * (g + u), total - 1);
      const int c = e / rows, r = e - c * rows;
      so[u] = (uint32_t)(c * lds + r);
      dofs[u] = (uint32_t)(c * ldd + r);
    }
    double2 v[NP > 0 ? NP : 1][B];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int u = 0; u < B; ++u) v[p][u] = ldc(J.src[p] + so[u]);
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (base + 256 * (g + u) >= total) break;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        re += J.coef[p].re * v[p][u].x - J.coef[p].im * v[p][u].y;
        im += J.coef[p].re * v[p][u].y + J.coef[p].im * v[p][u].x;
      }
      stc(J.dst + dofs[u], re, im);
    }
  }
}

// tile `tile` of a job list (jobs ordered by tile_begin), thread t of 256,
// B elements of the thread in flight at once
template <int B>
__device__ __forceinline__ void assemble_one(const AsmJob* __restrict__ jobs, int njobs, int tile, int t) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  const AsmJob& J = jobs[lo];
  const int base = (tile - J.tile_begin) * kAsmTile + t;
  switch (J.npieces) {  // 0: a block of zeros
    case 0:
      assemble_tile<0, B>(J, base);
      break;
    case 1:
      assemble_tile<1, B>(J, base);
      break;
    case 2:
      assemble_tile<2, B>(J, base);
      break;
    default:
      assemble_tile<3, B>(J, base);
  }
}

constexpr int kGjeNb = 16;  // panel width
constexpr int kGjeMaxN = 1024; // largest block order: the panel kernel holds 2 rows per thread (N_i <= 512)

constexpr int kGjePivStride = 84;  // ints per step: count, 2 NB destinations, 2 NB sources, NB pivot rows
constexpr int kRhsMaxN16 = 608;    // largest order whose 16-column right-hand-side tile fits in LDS
constexpr int kRhsMaxN10 = 1008;   // and a 10-column tile (157.5 KiB of the 160 KiB)

// one matrix W = [D | right-hand sides] (n x ncol, ld n) reduced to [. | D^{-1} rhs]
struct GjeDesc {
  cplx* W;
  cplx* M1;   // scratch ceil(n/NB) x NB x NB: inverse of each step's pivot block
  int* piv;   // scratch ceil(n/NB) x kGjePivStride: each step's row interchanges
  int* info;  // set to (global column + 1) on an exactly zero pivot
  int n, ncol;
};

// y = g - U1 x1 - U2 x2 (back substitution of the cyclic reduction, batched)
// Y = G - U1 X1 - U2 X2 with r right-hand-side columns (ld n for G and Y,
// m1 for X1, m2 for X2)
struct GemvDesc {
  const cplx* U1;  // n x m1, ld n
  const cplx* U2;  // n x m2, ld n
  const cplx* g;   // n x r
  const cplx* x1;  // m1 x r
  const cplx* x2;  // m2 x r
  cplx* y;         // n x r
  int n, m1, m2, r;
};

void gje_init();
void launch_gje_panel(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st);
// step k on columns [min(k + NB + lo, n), k + NB + hi) of the diagonal
// blocks (hi may exceed n); with max_col > 0 (orders up to the limit
// gje_step_fits checks) the range runs on through the right-hand-side
// columns, up to ncol, and max_col / max_rhs bound ncol and ncol - n
void launch_gje_update(const GjeDesc* d, int nbatch, int k, int max_n, int lo, int hi, hipStream_t st,
                       int max_col = 0, int max_rhs = 0);
// panel k and the update of step k - 16 in one launch (orders up to the
// limit gje_step_fits checks); max_col > 0 as for launch_gje_update
bool gje_step_fits(int max_n);
void launch_gje_step(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st, int max_col = 0,
                     int max_rhs = 0);
// workgroups of the largest launch_gje_step of a level (one fits a compute unit)
int gje_step_max_blocks(int nbatch, int max_n, int max_col, int max_rhs);
// right-hand-side replay of steps [s0, s1); max_blocks > 0 caps the grid
void launch_gje_premul(const GjeDesc* d, int nbatch, int max_n, hipStream_t st);
// narrow: 8-column tiles at every order (else 16 up to kRhsMaxN16)
void launch_gje_rhs(const GjeDesc* d, int nbatch, int max_rhs, int max_n, int s0, int s1, int max_blocks,
                    hipStream_t st, bool narrow = false);
void launch_gemv_step(const GemvDesc* d, int nbatch, int max_n, int max_r, hipStream_t st);

}  // namespace mlh

namespace mlh {

// Blocked Householder least squares of one layer (Sec. 3.2): the augmented
// matrix A = [S | RHS] (M x (c + ncol), ld M, M = m + c) with S = [Q; mu I]
// is reduced panel by panel (WY form), then R X = (Q^H RHS)[0:c] is solved
// by back substitution; X overwrites the top c rows of RHS.
constexpr int kHqNb = 16;
constexpr int kHqCols = 32;
constexpr int kHqMaxRows = 512;  // M  (LDS holds an M x 16 panel)
constexpr int kHqRhsSmallRows = 384;  // layers up to this M take the lighter right-hand-side kernel
constexpr int kHqMaxC = 256;     // c  (proxy plus Bragg unknowns of one layer)

struct HqDesc {
  cplx* A;
  cplx* T;    // scratch ceil(c/16) x 16 x 16: block reflector factor T of each panel
  double mu_rel;
  int m, c, ncol;
};

void launch_hq_prep(const HqDesc* d, int n, hipStream_t st);
// with asm_t1 > asm_t0 the launch also assembles tiles [asm_t0, asm_t1) of
// asm_jobs (work independent of the layer solves)
void launch_hq_panel(const HqDesc* d, int n, int k, hipStream_t st, const AsmJob* asm_jobs = nullptr,
                     int asm_njobs = 0, int asm_t0 = 0, int asm_t1 = 0);
// One launch over both layer size classes: descs [0, n_small) have at most
// kHqRhsSmallRows rows and take row_blocks (3 or 4) 16-row blocks per
// wavefront, descs [n_small, n_small + n_large) always 4; max_c and max_ncol
// are maxima over both classes
void launch_hq_update(const HqDesc* d, int n_small, int n_large, int k, int max_c, hipStream_t st,
                      int row_blocks = 3);
void launch_hq_rhs(const HqDesc* d, int n_small, int n_large, int max_ncol, int max_c, hipStream_t st,
                   int row_blocks = 3);

}  // namespace mlh
