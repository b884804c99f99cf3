// Host side of the C ABI declared in include/mlh.h: argument validation,
// quadrature geometry (Sec. 2.5), device memory layout, and the launch
// sequence of the fill, least-squares, Schur and sweep phases (Sec. 2-3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlh.h"
#include "../../include/mlh_debug.h"
#include "alpert_rule.inc"
#include "internal.hpp"

using namespace mlh;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static mlh_status fail(mlh_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

#define MLH_TRY(expr)                 \
  do {                                \
    mlh_status s_ = (expr);           \
    if (s_ != MLH_OK) return s_;      \
  } while (0)

extern "C" const char* mlh_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct mlh_ctx_s {
  int device;
  hipStream_t stream;
  char* scratch;  // this device's fixed workspace (allocation-free solve)
};

extern "C" mlh_status mlh_ctx_create(int32_t device, void* hip_stream, mlh_ctx* out) {
  if (!out) return fail(MLH_E_INVALID_ARG, "mlh_ctx_create: out is NULL");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MLH_E_INVALID_ARG, "mlh_ctx_create: no such device");
  HIP_TRY(hipSetDevice(device));
  gje_init();
  char* scratch = nullptr;
  HIP_TRY(scratch_address(device, &scratch));
  *out = new mlh_ctx_s{device, (hipStream_t)hip_stream, scratch};
  return MLH_OK;
}

extern "C" mlh_status mlh_ctx_destroy(mlh_ctx ctx) {
  delete ctx;
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// host geometry of one smooth interface
// ---------------------------------------------------------------------------
namespace {

struct FourierProfile {
  std::vector<double> ca, sa, om;

  double f(double x) const {
    double s = 0.0;
    for (size_t m = 0; m < om.size(); ++m) s += ca[m] * std::cos(om[m] * x) + sa[m] * std::sin(om[m] * x);
    return s;
  }
  double fp(double x) const {
    double s = 0.0;
    for (size_t m = 0; m < om.size(); ++m) s += om[m] * (-ca[m] * std::sin(om[m] * x) + sa[m] * std::cos(om[m] * x));
    return s;
  }
  // f(x + h) - f(x) from product formulas
  double diff(double x, double h) const {
    double s = 0.0;
    for (size_t m = 0; m < om.size(); ++m) {
      const double sh = std::sin(0.5 * om[m] * h), mid = om[m] * (x + 0.5 * h);
      s += -2.0 * ca[m] * std::sin(mid) * sh + 2.0 * sa[m] * std::cos(mid) * sh;
    }
    return s;
  }
  // f(x + h) - f(x) - h f'(x), mode by mode
  double rem(double x, double h) const {
    double s = 0.0;
    for (size_t m = 0; m < om.size(); ++m) {
      const double u = om[m] * h;
      const double su = std::sin(0.5 * u);
      const double cm1 = -2.0 * su * su;
      double smu;
      if (std::fabs(u) < 0.5) {  // sin u - u by its Taylor series
        const double u2 = u * u;
        double term = -u * u2 / 6.0, acc = 0.0;
        for (int k = 0; k < 12; ++k) {
          acc += term;
          term *= -u2 / ((2.0 * k + 4.0) * (2.0 * k + 5.0));
        }
        smu = acc;
      } else {
        smu = std::sin(u) - u;
      }
      const double c = std::cos(om[m] * x), s_ = std::sin(om[m] * x);
      s += ca[m] * (c * cm1 - s_ * smu) + sa[m] * (s_ * cm1 + c * smu);
    }
    return s;
  }
};

struct HostCurve {
  int N = 0;
  bool cornered = false;
  double y0 = 0.0;
  FourierProfile prof;
  std::vector<double> vx, vy;                            // cornered: vertices (absolute y)
  std::vector<double> x, y, nx, ny, w;                   // y relative to y0
  std::vector<int> seg_lo, seg_len;                      // cornered: segment of each node
  std::vector<double> ar2, and_, anpd, ann, acw, at;     // Alpert aux invariants, N x 30

  // absolute height of the interface at abscissa x in the unit cell
  double height(double xx) const {
    if (!cornered) return y0 + prof.f(xx);
    size_t c = 0;
    while (c + 2 < vx.size() && xx > vx[c + 1]) ++c;
    const double t = (xx - vx[c]) / (vx[c + 1] - vx[c]);
    return vy[c] + t * (vy[c + 1] - vy[c]);
  }
};

// Kress grading (Sec. 2.5): w(s) = 2 pi v(s)^q/(v(s)^q + v(2 pi - s)^q).
// Returns w, its complement 2 pi - w (formed from v(2 pi - s)^q so that it
// keeps its relative accuracy near s = 2 pi) and w'.
struct Kress {
  double w, wc, wp;
};
Kress kress(double s, double q) {
  auto v = [q](double t) {
    const double u = (kPi - t) / kPi;
    return (1.0 / q - 0.5) * u * u * u + (t - kPi) / (q * kPi) + 0.5;
  };
  auto vp = [q](double t) {
    const double u = (kPi - t) / kPi;
    return -(3.0 / kPi) * (1.0 / q - 0.5) * u * u + 1.0 / (q * kPi);
  };
  const double va = v(s), vb = v(2.0 * kPi - s);
  const double A = std::pow(va, q), B = std::pow(vb, q);
  const double Ap = q * std::pow(va, q - 1.0) * vp(s);
  const double Bp = -q * std::pow(vb, q - 1.0) * vp(2.0 * kPi - s);
  const double den = A + B;
  return {2.0 * kPi * A / den, 2.0 * kPi * B / den, 2.0 * kPi * (Ap * B - A * Bp) / (den * den)};
}

// Cornered interface: straight segments between consecutive vertices, each
// with its own Kress-graded trapezoid rule s_j = 2 pi (j - 1/2)/n (midpoints).
// A node is placed from its nearer corner so that its distance to that corner
// survives rounding.  The Alpert correction runs per segment, periodic in s
// with no phase; on a straight segment the separation of two of its points is
// (w(s_m) - w(s))/(2 pi) times the chord, orthogonal to the normal.
void build_polygon_curve(const mlh_interface& in, HostCurve& c) {
  c.cornered = true;
  c.y0 = in.y0;
  c.vx.assign(in.vx, in.vx + in.n_vert);
  c.vy.assign(in.vy, in.vy + in.n_vert);
  const int nseg = in.n_vert - 1;
  int N = 0;
  for (int g = 0; g < nseg; ++g) N += in.seg_nodes[g];
  c.N = N;
  c.x.resize(N);
  c.y.resize(N);
  c.nx.resize(N);
  c.ny.resize(N);
  c.w.resize(N);
  c.seg_lo.resize(N);
  c.seg_len.resize(N);
  const size_t na = (size_t)N * kAlpertAux;
  c.ar2.assign(na, 0.0);
  c.and_.assign(na, 0.0);
  c.anpd.assign(na, 0.0);
  c.ann.assign(na, 1.0);
  c.acw.resize(na);
  c.at.resize(na);
  const double q = in.q;
  int lo = 0;
  for (int g = 0; g < nseg; ++g) {
    const int n = in.seg_nodes[g];
    const double dx = c.vx[g + 1] - c.vx[g], dy = c.vy[g + 1] - c.vy[g];
    const double L = std::hypot(dx, dy);
    const double h = 2.0 * kPi / n;
    for (int j = 0; j < n; ++j) {
      const double sj = h * (j + 0.5);
      const Kress K = kress(sj, q);
      const int i = lo + j;
      if (sj < kPi) {
        c.x[i] = c.vx[g] + K.w / (2.0 * kPi) * dx;
        c.y[i] = (c.vy[g] - c.y0) + K.w / (2.0 * kPi) * dy;
      } else {
        c.x[i] = c.vx[g + 1] - K.wc / (2.0 * kPi) * dx;
        c.y[i] = (c.vy[g + 1] - c.y0) - K.wc / (2.0 * kPi) * dy;
      }
      c.nx[i] = dy / L;
      c.ny[i] = -dx / L;
      c.w[i] = L / n * K.wp;
      c.seg_lo[i] = lo;
      c.seg_len[i] = n;
      for (int qa = 0; qa < kAlpertAux; ++qa) {
        const int kq = qa % kAlpertJ;
        const double sg = qa < kAlpertJ ? 1.0 : -1.0;
        const double t = j + sg * kAlpertChi[kq];  // segment-local index units
        double sa = std::fmod(h * (t + 0.5), 2.0 * kPi);
        if (sa < 0) sa += 2.0 * kPi;
        const Kress Ka = kress(sa, q);
        const double dw = (sj >= kPi && sa >= kPi) ? Ka.wc - K.wc : K.w - Ka.w;
        const double sep = dw / (2.0 * kPi) * L;
        const size_t o = (size_t)i * kAlpertAux + qa;
        c.ar2[o] = sep * sep;
        c.acw[o] = kAlpertW[kq];
        c.at[o] = t;
      }
    }
    lo += n;
  }
}

void build_fourier_curve(const mlh_interface& in, double d, HostCurve& c) {
  c.N = in.n_nodes;
  c.y0 = in.y0;
  c.prof.ca.assign(in.cos_coef, in.cos_coef + in.n_modes);
  c.prof.sa.assign(in.sin_coef, in.sin_coef + in.n_modes);
  c.prof.om.resize(in.n_modes);
  for (int m = 0; m < in.n_modes; ++m) c.prof.om[m] = 2.0 * kPi * (m + 1) / d;
  const int N = c.N;
  const double hx = d / N;
  c.x.resize(N);
  c.y.resize(N);
  c.nx.resize(N);
  c.ny.resize(N);
  c.w.resize(N);
  for (int j = 0; j < N; ++j) {
    const double x = -0.5 * d + hx * (j + 0.5);
    const double fp = c.prof.fp(x);
    const double nu = std::sqrt(1.0 + fp * fp);
    c.x[j] = x;
    c.y[j] = c.prof.f(x);
    c.nx[j] = fp / nu;
    c.ny[j] = -1.0 / nu;
    c.w[j] = hx * nu;
  }
  // auxiliary nodes s_m +- chi_k h of the Alpert correction, with separations
  // formed without cancellation
  const size_t na = (size_t)N * kAlpertAux;
  c.ar2.resize(na);
  c.and_.resize(na);
  c.anpd.resize(na);
  c.ann.resize(na);
  c.acw.resize(na);
  c.at.resize(na);
  for (int m = 0; m < N; ++m) {
    const double xm = c.x[m];
    const double fm = c.prof.fp(xm);
    const double num = std::sqrt(1.0 + fm * fm);
    for (int q = 0; q < kAlpertAux; ++q) {
      const int kq = q % kAlpertJ;
      const double sg = q < kAlpertJ ? 1.0 : -1.0;
      const double chi = kAlpertChi[kq];
      const double dx = sg * chi * hx;
      const double xs = xm + dx;
      const double fs = c.prof.fp(xs);
      const double nus = std::sqrt(1.0 + fs * fs);
      const double df = c.prof.diff(xm, dx);
      const size_t i = (size_t)m * kAlpertAux + q;
      c.ar2[i] = dx * dx + df * df;
      c.and_[i] = c.prof.rem(xm, dx) / num;
      c.anpd[i] = -c.prof.rem(xs, -dx) / nus;
      c.ann[i] = (fm * fs + 1.0) / (num * nus);
      c.acw[i] = kAlpertW[kq] * hx * nus;
      c.at[i] = m + sg * chi;
    }
  }
}

// f(0..n-1) on up to 16 host threads (the calling thread included); f must
// touch only state of its own index
template <class F>
static void parallel_for(int n, F f) {
  const int nt = std::max(1, std::min({16, (int)std::thread::hardware_concurrency(), n}));
  std::vector<std::thread> pool;
  for (int w = 1; w < nt; ++w)
    pool.emplace_back([&f, w, nt, n]() {
      for (int i = w; i < n; i += nt) f(i);
    });
  for (int i = 0; i < n; i += nt) f(i);
  for (std::thread& th : pool) th.join();
}

// Device state solves run in: the workspace, reused across calls that fit
// it, and the captured launch sequence, replayed while the batch shape and
// the workspace stay the same (only the descriptor contents change).
struct Runner {
  char* wmem = nullptr;
  size_t wbytes = 0;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> g_sig;
  hipStream_t cap_stream = nullptr;
  hipStream_t aux_stream = nullptr;  // second stream of the Gauss-Jordan look-ahead
  std::vector<hipEvent_t> evpool;    // its dependency events
  int num_cu = 0;                    // compute units of the device
  // teardown: errors here leave nothing to recover
  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (aux_stream) (void)hipStreamDestroy(aux_stream);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    if (wmem) (void)hipFree(wmem);
    gexec = nullptr;
    cap_stream = aux_stream = nullptr;
    evpool.clear();
    wmem = nullptr;
    wbytes = 0;
  }
};

// simple bump allocator over one device arena
struct Arena {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  size_t reserve(size_t bytes) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return o;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// stack
// ---------------------------------------------------------------------------
struct mlh_stack_s {
  mlh_ctx ctx = nullptr;
  // device scratch of mlh_adjoint, kept between calls and grown on demand:
  // its buffers, their job tables, a shape-gradient pass, its contractions
  std::pair<char*, size_t> adj_buf[4] = {};
  mlh_tuning tune{300, 3, 16, 1, 8};  // launch choices (mlh_stack_set_tuning / mlh_stack_autotune)
  double flux_tol = 0.0;           // > 0: a solve whose flux error exceeds it reports MLH_E_ACCURACY
  int I = 0, P = 0, Mw = 0, Mud = 0, K = 0, nK = 0;
  double d = 0, yU = 0, yD = 0, R = 0, mu = 1e-14;
  std::vector<double> k;
  std::vector<HostCurve> curves;
  std::vector<int> N, n;
  std::vector<double> centre;  // proxy circle centre heights per layer

  char* dmem = nullptr;
  size_t dbytes = 0;
  // device geometry
  std::vector<double*> gx, gy, gnx, gny, gw;
  std::vector<double*> ar2, and_, anpd, ann, acw, at;
  std::vector<int*> seg_lo, seg_len;  // cornered interfaces only (else null)
  std::vector<double*> wall_x, wall_y;  // per layer, y relative to centre
  double* ud_x = nullptr;
  double* ud_y = nullptr;  // zeros
  std::vector<double*> px, py, pnx, pny;  // per layer, y relative to centre
  // pieces
  std::vector<cplx*> A_self, A_up, A_dn, B_own, B_below, C_own, C_above, Q;
  cplx* Z_U = nullptr;
  cplx* Z_D = nullptr;
  cplx* V_U = nullptr;
  cplx* V_D = nullptr;
  // fill job tables on the device
  FillJob* d_fill = nullptr;
  int n_fill = 0, fill_tiles = 0;
  SelfJob* d_self = nullptr;
  int n_self = 0, self_tiles = 0;
  AlpertJob* d_alp = nullptr;
  int n_alp = 0, alp_blocks = 0;

  // workspace views of the first angle of the last inspection solve
  std::vector<cplx*> dbg_R, dbg_S, dbg_RHS, dbg_eta;

  // host copies of the fill job tables (merged into batch launches)
  std::vector<FillJob> h_fill;
  std::vector<SelfJob> h_self;
  std::vector<AlpertJob> h_alp;

  Runner run;  // workspace and captured launch sequence of this stack's solves
};

static size_t cbytes(size_t n) { return n * sizeof(cplx); }

static mlh_status validate(const mlh_stack_desc* D) {
  if (!D) return fail(MLH_E_INVALID_ARG, "desc is NULL");
  if (D->abi_version != MLH_ABI_VERSION) return fail(MLH_E_INVALID_ARG, "abi_version mismatch");
  if (D->I < 1) return fail(MLH_E_INVALID_ARG, "I must be >= 1");
  if (!D->iface || !D->k) return fail(MLH_E_INVALID_ARG, "iface or k is NULL");
  if (!(D->d > 0) || !std::isfinite(D->d)) return fail(MLH_E_INVALID_ARG, "period d must be positive");
  for (int i = 0; i <= D->I; ++i)
    if (!(D->k[i] > 0) || !std::isfinite(D->k[i])) return fail(MLH_E_INVALID_ARG, "wavenumbers must be positive");
  if (D->P < 1 || !(D->R > 0)) return fail(MLH_E_INVALID_ARG, "need P >= 1 and R > 0");
  if (D->M_w < 1 || D->K < 0) return fail(MLH_E_INVALID_ARG, "need M_w >= 1 and K >= 0");
  if (D->M_ud < 2 * D->K + 1) return fail(MLH_E_INVALID_ARG, "M_ud must be >= 2K+1 (aliasing of Rayleigh-Bloch orders)");
  if (D->ls_mu < 0 || !std::isfinite(D->ls_mu)) return fail(MLH_E_INVALID_ARG, "ls_mu must be >= 0");
  if (2 * D->M_w + 2 * D->M_ud + D->P + 2 * D->K + 1 > kHqMaxRows || D->P + 2 * D->K + 1 > kHqMaxC)
    return fail(MLH_E_UNSUPPORTED, "least-squares blocks too large: need 2 M_w + 2 M_ud + P + 2K + 1 <= 512 "
                                   "and P + 2K + 1 <= 256");
  const int nmin = 2 * (kAlpertA + 8) + 1;
  const int nmax = kGjeMaxN / 2;
  for (int i = 0; i < D->I; ++i) {
    const mlh_interface& f = D->iface[i];
    if (!std::isfinite(f.y0)) return fail(MLH_E_INVALID_ARG, "non-finite y0");
    int ntot = 0;
    if (f.kind == MLH_IFACE_FOURIER) {
      if (f.n_modes < 0 || (f.n_modes > 0 && (!f.cos_coef || !f.sin_coef)))
        return fail(MLH_E_INVALID_ARG, "Fourier coefficients missing");
      if (f.n_nodes < nmin)
        return fail(MLH_E_INVALID_ARG, "each interface needs at least " + std::to_string(nmin) + " nodes");
      ntot = f.n_nodes;
    } else if (f.kind == MLH_IFACE_POLYGON) {
      if (f.n_vert < 2 || !f.vx || !f.vy || !f.seg_nodes)
        return fail(MLH_E_INVALID_ARG, "polygon interface needs n_vert >= 2, vx, vy and seg_nodes");
      if (!(f.q >= 2.0) || !std::isfinite(f.q)) return fail(MLH_E_INVALID_ARG, "grading exponent q must be >= 2");
      const double tol = 1e-12 * D->d;
      if (std::fabs(f.vx[0] + 0.5 * D->d) > tol || std::fabs(f.vx[f.n_vert - 1] - 0.5 * D->d) > tol)
        return fail(MLH_E_INVALID_ARG, "polygon must run from x = -d/2 to x = d/2");
      if (!(std::fabs(f.vy[0] - f.vy[f.n_vert - 1]) <= tol))
        return fail(MLH_E_INVALID_ARG, "polygon must be periodic: vy[0] == vy[n_vert-1]");
      for (int c = 0; c + 1 < f.n_vert; ++c) {
        if (!std::isfinite(f.vy[c]) || !(f.vx[c + 1] > f.vx[c]))
          return fail(MLH_E_INVALID_ARG, "polygon vertices must have finite, strictly increasing x");
        if (f.seg_nodes[c] < nmin)
          return fail(MLH_E_INVALID_ARG, "each polygon segment needs at least " + std::to_string(nmin) + " nodes");
        ntot += f.seg_nodes[c];
      }
    } else {
      return fail(MLH_E_INVALID_ARG, "unknown interface kind");
    }
    if (ntot > nmax)
      return fail(MLH_E_UNSUPPORTED, "at most " + std::to_string(nmax) + " nodes per interface are supported");
  }
  return MLH_OK;
}

// interfaces must be ordered and separated, radiation lines clear, proxy
// circles must enclose their layer cell
static mlh_status check_geometry(mlh_stack_s* s) {
  const int G = 512;
  std::vector<double> lo(s->I), hi(s->I);
  std::vector<std::vector<double>> prof(s->I, std::vector<double>(G + 1));
  for (int i = 0; i < s->I; ++i) {
    lo[i] = 1e300;
    hi[i] = -1e300;
    for (int g = 0; g <= G; ++g) {
      const double x = -0.5 * s->d + s->d * g / G;
      const double y = s->curves[i].height(x);
      prof[i][g] = y;
      lo[i] = std::min(lo[i], y);
      hi[i] = std::max(hi[i], y);
    }
    for (double vy : s->curves[i].vy) {  // corners between grid points
      lo[i] = std::min(lo[i], vy);
      hi[i] = std::max(hi[i], vy);
    }
  }
  for (int i = 0; i + 1 < s->I; ++i)
    for (int g = 0; g <= G; ++g)
      if (!(prof[i + 1][g] < prof[i][g]))
        return fail(MLH_E_GEOMETRY, "interfaces " + std::to_string(i + 1) + " and " + std::to_string(i + 2) + " cross");
  if (!(s->yU > hi[0])) return fail(MLH_E_GEOMETRY, "y_U must lie above the first interface");
  if (!(s->yD < lo[s->I - 1])) return fail(MLH_E_GEOMETRY, "y_D must lie below the last interface");
  for (int j = 0; j <= s->I; ++j) {
    const double top = j == 0 ? s->yU : hi[j - 1];
    const double bot = j == s->I ? s->yD : lo[j];
    const double c = s->centre[j];
    const double r = std::hypot(0.5 * s->d, std::max(top - c, c - bot));
    if (!(s->R > r))
      return fail(MLH_E_GEOMETRY, "proxy circle of layer " + std::to_string(j + 1) + " does not enclose its cell");
  }
  return MLH_OK;
}

static void build_fill_tables(mlh_stack_s* s, std::vector<FillJob>& fj, std::vector<SelfJob>& sj,
                              std::vector<AlpertJob>& aj) {
  const int I = s->I;
  const double d = s->d;
  int tiles = 0;
  auto add = [&](FillJob J) {
    const int tm = J.kind == kFillPair ? kSelfTile : kFillTileM, tn = J.kind == kFillPair ? kSelfTile : kFillTileN;
    J.tiles_m = (J.Mt + tm - 1) / tm;
    J.tile_begin = tiles;
    tiles += J.tiles_m * ((J.Ns + tn - 1) / tn);
    fj.push_back(J);
  };
  auto curve_src = [&](FillJob& J, int i) {
    J.sx = s->gx[i];
    J.sy = s->gy[i];
    J.snx = s->gnx[i];
    J.sny = s->gny[i];
    J.sw = s->gw[i];
    J.Ns = s->N[i];
  };
  auto curve_tgt = [&](FillJob& J, int i) {
    J.tx = s->gx[i];
    J.ty = s->gy[i];
    J.tnx = s->gnx[i];
    J.tny = s->gny[i];
    J.Mt = s->N[i];
  };
  auto proxy_src = [&](FillJob& J, int layer) {
    J.sx = s->px[layer];
    J.sy = s->py[layer];
    J.snx = s->pnx[layer];
    J.sny = s->pny[layer];
    J.sw = nullptr;
    J.Ns = s->P;
  };
  auto three = [&](FillJob& J, cplx* base, size_t piece_elems) {
    J.npieces = 3;
    for (int l = 0; l < 3; ++l) {
      J.tshift[l] = 0.0;
      J.sshift[l] = (l - 1) * d;
      J.out[l] = base + l * piece_elems;
    }
  };
  // neighbour blocks A_{i,i+1} = -[...]^{k_{i+1}}, A_{i+1,i} = +[...]^{k_{i+1}},
  // both from one job: A_{i+1,i} copy l is A_{i,i+1} copy -l transposed
  for (int i = 0; i + 1 < I; ++i) {
    FillJob J{};
    curve_tgt(J, i);
    curve_src(J, i + 1);
    J.kind = kFillPair;
    J.k = s->k[i + 1];
    J.scale = -1.0;
    J.dy0 = s->curves[i].y0 - s->curves[i + 1].y0;
    J.ld = s->n[i];
    three(J, s->A_up[i], (size_t)s->n[i] * s->n[i + 1]);
    J.ld_t = s->n[i + 1];
    J.tw = s->gw[i];
    J.scale_t = 1.0;
    for (int l = 0; l < 3; ++l) J.out_t[l] = s->A_dn[i] + (size_t)l * s->n[i + 1] * s->n[i];
    add(J);
  }
  // proxy blocks B_{i,i} (layer above) and B_{i,i+1} (layer below, negated)
  for (int i = 0; i < I; ++i) {
    for (int side = 0; side < 2; ++side) {
      const int layer = i + side;
      FillJob J{};
      curve_tgt(J, i);
      proxy_src(J, layer);
      J.kind = kFillProxy;
      J.k = s->k[layer];
      J.scale = side ? -1.0 : 1.0;
      J.dy0 = s->curves[i].y0 - s->centre[layer];
      J.ld = s->n[i];
      J.npieces = 1;
      J.out[0] = side ? s->B_below[i] : s->B_own[i];
      add(J);
    }
  }
  // wall blocks: C (targets x + 2d and x - d) and Q (x + d and x), normal (1, 0)
  for (int j = 0; j <= I; ++j) {
    for (int side = 0; side < 2; ++side) {
      const int src = side == 0 ? j : j - 1;  // C_own: Gamma_j ; C_above: Gamma_{j-1}
      if (src < 0 || src >= I) continue;
      FillJob J{};
      J.tx = s->wall_x[j];
      J.ty = s->wall_y[j];
      J.tnx = nullptr;
      J.tny = nullptr;
      J.cnx = 1.0;
      J.cny = 0.0;
      J.Mt = s->Mw;
      curve_src(J, src);
      J.kind = kFillLayerPotential;
      J.k = s->k[j];
      J.scale = 1.0;
      J.dy0 = s->centre[j] - s->curves[src].y0;
      J.ld = 2 * s->Mw;
      J.npieces = 2;
      const size_t pe = (size_t)2 * s->Mw * s->n[src];
      cplx* base = side == 0 ? s->C_own[j] : s->C_above[j];
      J.tshift[0] = 2 * d;
      J.tshift[1] = -d;
      J.sshift[0] = J.sshift[1] = 0.0;
      J.out[0] = base;
      J.out[1] = base + pe;
      add(J);
    }
    FillJob J{};
    J.tx = s->wall_x[j];
    J.ty = s->wall_y[j];
    J.cnx = 1.0;
    J.cny = 0.0;
    J.Mt = s->Mw;
    proxy_src(J, j);
    J.kind = kFillProxy;
    J.k = s->k[j];
    J.scale = 1.0;
    J.dy0 = 0.0;
    J.ld = 2 * s->Mw;
    J.npieces = 2;
    J.tshift[0] = d;
    J.tshift[1] = 0.0;
    J.sshift[0] = J.sshift[1] = 0.0;
    J.out[0] = s->Q[j];
    J.out[1] = s->Q[j] + (size_t)2 * s->Mw * s->P;
    add(J);
  }
  // radiation lines: Z_U / Z_D (3 copies) and V_U / V_D, normal (0, 1)
  for (int side = 0; side < 2; ++side) {
    const int ci = side == 0 ? 0 : I - 1;
    const int layer = side == 0 ? 0 : I;
    const double yline = side == 0 ? s->yU : s->yD;
    FillJob J{};
    J.tx = s->ud_x;
    J.ty = s->ud_y;
    J.cnx = 0.0;
    J.cny = 1.0;
    J.Mt = s->Mud;
    curve_src(J, ci);
    J.kind = kFillLayerPotential;
    J.k = s->k[layer];
    J.scale = 1.0;
    J.dy0 = yline - s->curves[ci].y0;
    J.ld = 2 * s->Mud;
    three(J, side == 0 ? s->Z_U : s->Z_D, (size_t)2 * s->Mud * s->n[ci]);
    add(J);
    FillJob V{};
    V.tx = s->ud_x;
    V.ty = s->ud_y;
    V.cnx = 0.0;
    V.cny = 1.0;
    V.Mt = s->Mud;
    proxy_src(V, layer);
    V.kind = kFillProxy;
    V.k = s->k[layer];
    V.scale = 1.0;
    V.dy0 = yline - s->centre[layer];
    V.ld = 2 * s->Mud;
    V.npieces = 1;
    V.out[0] = side == 0 ? s->V_U : s->V_D;
    add(V);
  }
  s->fill_tiles = tiles;
  // self blocks and Alpert corrections
  int st = 0, ab = 0;
  for (int i = 0; i < I; ++i) {
    SelfJob S{};
    S.x = s->gx[i];
    S.y = s->gy[i];
    S.nx = s->gnx[i];
    S.ny = s->gny[i];
    S.w = s->gw[i];
    S.seg_lo = s->seg_lo[i];
    S.seg_len = s->seg_len[i];
    S.ka = s->k[i];
    S.kb = s->k[i + 1];
    S.d = d;
    S.N = s->N[i];
    const size_t pe = (size_t)s->n[i] * s->n[i];
    for (int l = 0; l < 3; ++l) S.out[l] = s->A_self[i] + l * pe;
    S.tiles_m = (S.N + kSelfTile - 1) / kSelfTile;
    S.tile_begin = st;
    st += S.tiles_m * (S.tiles_m + 1) / 2;
    sj.push_back(S);
    AlpertJob A{};
    A.r2 = s->ar2[i];
    A.nd = s->and_[i];
    A.npd = s->anpd[i];
    A.nn = s->ann[i];
    A.cw = s->acw[i];
    A.t = s->at[i];
    A.seg_lo = s->seg_lo[i];
    A.seg_len = s->seg_len[i];
    A.colw = s->seg_lo[i] ? s->gw[i] : nullptr;
    A.ka = s->k[i];
    A.kb = s->k[i + 1];
    for (int l = 0; l < 3; ++l) A.out[l] = S.out[l];
    A.N = s->N[i];
    A.block_begin = ab;
    ab += A.N;
    aj.push_back(A);
  }
  s->self_tiles = st;
  s->alp_blocks = ab;
}

static mlh_status run_fills(mlh_stack_s* s) {
  hipStream_t st = s->ctx->stream;
  launch_self(s->d_self, s->n_self, s->self_tiles, kAlpertA, st);
  HIP_TRY(hipGetLastError());
  launch_alpert(s->d_alp, s->n_alp, s->alp_blocks, kAlpertA, st);
  HIP_TRY(hipGetLastError());
  launch_fill(s->d_fill, s->n_fill, s->fill_tiles, st);
  HIP_TRY(hipGetLastError());
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_create(mlh_ctx ctx, const mlh_stack_desc* D, mlh_stack* out) {
  if (!ctx || !out) return fail(MLH_E_INVALID_ARG, "mlh_stack_create: NULL argument");
  MLH_TRY(validate(D));
  mlh_stack_s* s = new mlh_stack_s();
  s->ctx = ctx;
  s->I = D->I;
  s->P = D->P;
  s->Mw = D->M_w;
  s->Mud = D->M_ud;
  s->K = D->K;
  s->nK = 2 * D->K + 1;
  s->d = D->d;
  s->yU = D->y_U;
  s->yD = D->y_D;
  s->R = D->R;
  s->mu = D->ls_mu > 0 ? D->ls_mu : 1e-14;
  s->k.assign(D->k, D->k + D->I + 1);
  const int I = s->I;
  s->curves.resize(I);
  s->N.resize(I);
  s->n.resize(I);
  // the curves, with their Alpert auxiliary invariants, on host threads
  parallel_for(I, [&](int i) {
    if (D->iface[i].kind == MLH_IFACE_POLYGON)
      build_polygon_curve(D->iface[i], s->curves[i]);
    else
      build_fourier_curve(D->iface[i], s->d, s->curves[i]);
  });
  for (int i = 0; i < I; ++i) {
    s->N[i] = s->curves[i].N;
    s->n[i] = 2 * s->N[i];
    // strongly graded nodes of adjacent segments (also across x = +-d/2)
    // must stay distinct in float64
    const HostCurve& c = s->curves[i];
    if (c.cornered) {
      for (int a = 0; a < c.N; ++a)
        for (int b = 0; b < c.N; ++b)
          for (int l = -1; l <= 1; ++l) {
            if (l == 0 && a == b) continue;
            const double ddx = c.x[a] - c.x[b] - l * s->d, ddy = c.y[a] - c.y[b];
            if (ddx * ddx + ddy * ddy == 0.0) {
              delete s;
              return fail(MLH_E_INVALID_ARG, "graded nodes of interface " + std::to_string(i + 1) +
                                                 " coincide in float64: lower q or the segment node counts");
            }
          }
    }
  }
  // proxy circle centres: middle of each layer's nominal extent
  s->centre.resize(I + 1);
  for (int j = 0; j <= I; ++j) {
    const double top = j == 0 ? s->yU : s->curves[j - 1].y0;
    const double bot = j == I ? s->yD : s->curves[j].y0;
    s->centre[j] = 0.5 * (top + bot);
  }
  mlh_status gs = check_geometry(s);
  if (gs != MLH_OK) {
    delete s;
    return gs;
  }
  // ---- device layout
  Arena ar;
  std::vector<size_t> o_geo(I), o_aux(I), o_wall(I + 1), o_prox(I + 1);
  for (int i = 0; i < I; ++i) o_geo[i] = ar.reserve(sizeof(double) * 5 * s->N[i]);
  for (int i = 0; i < I; ++i) o_aux[i] = ar.reserve(sizeof(double) * 6 * (size_t)s->N[i] * kAlpertAux);
  std::vector<size_t> o_seg(I, 0);
  for (int i = 0; i < I; ++i)
    if (s->curves[i].cornered) o_seg[i] = ar.reserve(sizeof(int) * 2 * s->N[i]);
  for (int j = 0; j <= I; ++j) o_wall[j] = ar.reserve(sizeof(double) * 2 * s->Mw);
  const size_t o_ud = ar.reserve(sizeof(double) * 2 * s->Mud);
  for (int j = 0; j <= I; ++j) o_prox[j] = ar.reserve(sizeof(double) * 4 * s->P);
  std::vector<size_t> o_as(I), o_au(I), o_ad(I), o_bo(I), o_bb(I), o_co(I + 1), o_ca(I + 1), o_q(I + 1);
  for (int i = 0; i < I; ++i) o_as[i] = ar.reserve(cbytes((size_t)3 * s->n[i] * s->n[i]));
  for (int i = 0; i + 1 < I; ++i) {
    o_au[i] = ar.reserve(cbytes((size_t)3 * s->n[i] * s->n[i + 1]));
    o_ad[i] = ar.reserve(cbytes((size_t)3 * s->n[i + 1] * s->n[i]));
  }
  for (int i = 0; i < I; ++i) {
    o_bo[i] = ar.reserve(cbytes((size_t)s->n[i] * s->P));
    o_bb[i] = ar.reserve(cbytes((size_t)s->n[i] * s->P));
  }
  for (int j = 0; j <= I; ++j) {
    if (j < I) o_co[j] = ar.reserve(cbytes((size_t)2 * 2 * s->Mw * s->n[j]));
    if (j > 0) o_ca[j] = ar.reserve(cbytes((size_t)2 * 2 * s->Mw * s->n[j - 1]));
    o_q[j] = ar.reserve(cbytes((size_t)2 * 2 * s->Mw * s->P));
  }
  const size_t o_zu = ar.reserve(cbytes((size_t)3 * 2 * s->Mud * s->n[0]));
  const size_t o_zd = ar.reserve(cbytes((size_t)3 * 2 * s->Mud * s->n[I - 1]));
  const size_t o_vu = ar.reserve(cbytes((size_t)2 * s->Mud * s->P));
  const size_t o_vd = ar.reserve(cbytes((size_t)2 * s->Mud * s->P));
  // job tables are sized after the pointers are known
  std::vector<FillJob> fj;
  std::vector<SelfJob> sj;
  std::vector<AlpertJob> aj;
  const size_t o_fill = ar.reserve(sizeof(FillJob) * (size_t)(2 * I + 2 * I + 3 * (I + 1) + 4 + 8));
  const size_t o_self = ar.reserve(sizeof(SelfJob) * I);
  const size_t o_alp = ar.reserve(sizeof(AlpertJob) * I);
  s->dbytes = ar.off;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&s->dmem, s->dbytes);
  if (e != hipSuccess) {
    delete s;
    return fail(e == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE, "stack allocation failed");
  }
  char* b = s->dmem;
  auto dp = [&](size_t o) { return reinterpret_cast<double*>(b + o); };
  auto cp = [&](size_t o) { return reinterpret_cast<cplx*>(b + o); };
  s->gx.resize(I);
  s->gy.resize(I);
  s->gnx.resize(I);
  s->gny.resize(I);
  s->gw.resize(I);
  s->ar2.resize(I);
  s->and_.resize(I);
  s->anpd.resize(I);
  s->ann.resize(I);
  s->acw.resize(I);
  s->at.resize(I);
  s->seg_lo.assign(I, nullptr);
  s->seg_len.assign(I, nullptr);
  std::vector<double> hbuf;
  hipStream_t st = ctx->stream;
  for (int i = 0; i < I; ++i) {
    const int N = s->N[i];
    double* g = dp(o_geo[i]);
    s->gx[i] = g;
    s->gy[i] = g + N;
    s->gnx[i] = g + 2 * N;
    s->gny[i] = g + 3 * N;
    s->gw[i] = g + 4 * N;
    const HostCurve& c = s->curves[i];
    hbuf.clear();
    for (auto* v : {&c.x, &c.y, &c.nx, &c.ny, &c.w}) hbuf.insert(hbuf.end(), v->begin(), v->end());
    HIP_TRY(hipMemcpy(g, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice));
    const size_t na = (size_t)N * kAlpertAux;
    double* a = dp(o_aux[i]);
    s->ar2[i] = a;
    s->and_[i] = a + na;
    s->anpd[i] = a + 2 * na;
    s->ann[i] = a + 3 * na;
    s->acw[i] = a + 4 * na;
    s->at[i] = a + 5 * na;
    hbuf.clear();
    for (auto* v : {&c.ar2, &c.and_, &c.anpd, &c.ann, &c.acw, &c.at}) hbuf.insert(hbuf.end(), v->begin(), v->end());
    HIP_TRY(hipMemcpy(a, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice));
    if (c.cornered) {
      int* sg = reinterpret_cast<int*>(b + o_seg[i]);
      s->seg_lo[i] = sg;
      s->seg_len[i] = sg + N;
      std::vector<int> ib(c.seg_lo);
      ib.insert(ib.end(), c.seg_len.begin(), c.seg_len.end());
      HIP_TRY(hipMemcpy(sg, ib.data(), ib.size() * sizeof(int), hipMemcpyHostToDevice));
    }
  }
  // walls: M_w Gauss-Legendre nodes on x = -d/2 between the layer's boundaries
  std::vector<double> gl_t(s->Mw), gl_w(s->Mw);
  {
    const int M = s->Mw;
    for (int i = 0; i < M; ++i) {  // Newton on P_M from the Chebyshev guess
      double t = std::cos(kPi * (i + 0.75) / (M + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= M; ++k) {
          const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        if (M == 1) {
          p1 = t;
          p0 = 1.0;
        }
        const double dp = M * (t * p1 - p0) / (t * t - 1.0);
        const double dt = p1 / dp;
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
      gl_t[M - 1 - i] = t;
    }
  }
  s->wall_x.resize(I + 1);
  s->wall_y.resize(I + 1);
  for (int j = 0; j <= I; ++j) {
    const double top = j == 0 ? s->yU : s->curves[j - 1].height(-0.5 * s->d);
    const double bot = j == I ? s->yD : s->curves[j].height(-0.5 * s->d);
    hbuf.assign(2 * s->Mw, -0.5 * s->d);
    for (int m = 0; m < s->Mw; ++m) hbuf[s->Mw + m] = bot + (top - bot) * 0.5 * (gl_t[m] + 1.0) - s->centre[j];
    double* w = dp(o_wall[j]);
    s->wall_x[j] = w;
    s->wall_y[j] = w + s->Mw;
    HIP_TRY(hipMemcpy(w, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  hbuf.assign(2 * s->Mud, 0.0);
  for (int m = 0; m < s->Mud; ++m) hbuf[m] = -0.5 * s->d + s->d * (m + 0.5) / s->Mud;
  s->ud_x = dp(o_ud);
  s->ud_y = s->ud_x + s->Mud;
  HIP_TRY(hipMemcpy(s->ud_x, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice));
  s->px.resize(I + 1);
  s->py.resize(I + 1);
  s->pnx.resize(I + 1);
  s->pny.resize(I + 1);
  for (int j = 0; j <= I; ++j) {
    hbuf.assign(4 * s->P, 0.0);
    for (int p = 0; p < s->P; ++p) {
      const double th = 2.0 * kPi * (p + 1) / s->P;
      hbuf[p] = s->R * std::cos(th);
      hbuf[s->P + p] = s->R * std::sin(th);
      hbuf[2 * s->P + p] = std::cos(th);
      hbuf[3 * s->P + p] = std::sin(th);
    }
    double* q = dp(o_prox[j]);
    s->px[j] = q;
    s->py[j] = q + s->P;
    s->pnx[j] = q + 2 * s->P;
    s->pny[j] = q + 3 * s->P;
    HIP_TRY(hipMemcpy(q, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  s->A_self.resize(I);
  s->A_up.assign(I, nullptr);
  s->A_dn.assign(I, nullptr);
  s->B_own.resize(I);
  s->B_below.resize(I);
  s->C_own.assign(I + 1, nullptr);
  s->C_above.assign(I + 1, nullptr);
  s->Q.resize(I + 1);
  for (int i = 0; i < I; ++i) {
    s->A_self[i] = cp(o_as[i]);
    if (i + 1 < I) {
      s->A_up[i] = cp(o_au[i]);
      s->A_dn[i] = cp(o_ad[i]);
    }
    s->B_own[i] = cp(o_bo[i]);
    s->B_below[i] = cp(o_bb[i]);
  }
  for (int j = 0; j <= I; ++j) {
    if (j < I) s->C_own[j] = cp(o_co[j]);
    if (j > 0) s->C_above[j] = cp(o_ca[j]);
    s->Q[j] = cp(o_q[j]);
  }
  s->Z_U = cp(o_zu);
  s->Z_D = cp(o_zd);
  s->V_U = cp(o_vu);
  s->V_D = cp(o_vd);
  build_fill_tables(s, fj, sj, aj);
  s->d_fill = reinterpret_cast<FillJob*>(b + o_fill);
  s->d_self = reinterpret_cast<SelfJob*>(b + o_self);
  s->d_alp = reinterpret_cast<AlpertJob*>(b + o_alp);
  s->n_fill = (int)fj.size();
  s->n_self = (int)sj.size();
  s->n_alp = (int)aj.size();
  HIP_TRY(hipMemcpy(s->d_fill, fj.data(), sizeof(FillJob) * fj.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->d_self, sj.data(), sizeof(SelfJob) * sj.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->d_alp, aj.data(), sizeof(AlpertJob) * aj.size(), hipMemcpyHostToDevice));
  s->h_fill = fj;
  s->h_self = sj;
  s->h_alp = aj;
  mlh_status fs = run_fills(s);
  if (fs == MLH_OK) {
    hipError_t e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) fs = fail(MLH_E_DEVICE, std::string("fill: ") + hipGetErrorString(e2));
  }
  if (fs != MLH_OK) {
    (void)hipFree(s->dmem);
    delete s;
    return fs;
  }
  *out = s;
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_refill(mlh_stack s) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  HIP_TRY(hipSetDevice(s->ctx->device));
  MLH_TRY(run_fills(s));
  HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_destroy(mlh_stack s) {
  if (!s) return MLH_OK;
  // teardown: errors here leave nothing to recover
  (void)hipSetDevice(s->ctx->device);
  if (s->dmem) (void)hipFree(s->dmem);
  for (auto& b : s->adj_buf)
    if (b.first) (void)hipFree(b.first);
  s->run.release();
  delete s;
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_info(mlh_stack s, int64_t* n_den, int64_t* n_tot, int64_t* device_bytes) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  int64_t nd = 0;
  for (int v : s->n) nd += v;
  if (n_den) *n_den = nd;
  if (n_tot) *n_tot = nd + (int64_t)(s->I + 1) * s->P + 2 * s->nK;
  if (device_bytes) *device_bytes = (int64_t)(s->dbytes + s->run.wbytes);
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
namespace {

inline cplx cx(double re, double im) { return cplx{re, im}; }
inline cplx cpow_alpha(double phase, int p) { return cplx{std::cos(p * phase), std::sin(p * phase)}; }

}  // namespace

static void layer_dims(const mlh_stack_s* s, int j, int& m, int& c, int& ncol) {
  const int I = s->I;
  const bool end = (j == 0 || j == I);
  m = 2 * s->Mw + (end ? 2 * s->Mud : 0);
  c = s->P + (end ? s->nK : 0);
  if (j == 0)
    ncol = s->n[0];
  else if (j == I)
    ncol = s->n[I - 1];
  else
    ncol = s->n[j - 1] + s->n[j];
}

// HIP-event timer for the profiling entry point
namespace {
struct EvTimer {
  hipStream_t st;
  std::vector<hipEvent_t> ev;
  std::vector<double*> dst;
  std::vector<int> pairs;     // index of start event per interval
  hipError_t err = hipSuccess;  // the first failure; collect() returns it
  void keep(hipError_t e) {
    if (err == hipSuccess) err = e;
  }
  void record() {
    hipEvent_t e = nullptr;
    const hipError_t ce = hipEventCreate(&e);
    keep(ce);
    if (ce == hipSuccess) keep(hipEventRecord(e, st));
    ev.push_back(e);
  }
  void begin(double* acc) {
    pairs.push_back((int)ev.size());
    dst.push_back(acc);
    record();
  }
  void end() { record(); }
  hipError_t collect() {
    keep(hipStreamSynchronize(st));
    for (size_t i = 0; i < pairs.size() && err == hipSuccess; ++i) {
      float ms = 0.f;
      keep(hipEventElapsedTime(&ms, ev[pairs[i]], ev[pairs[i] + 1]));
      *dst[i] += ms;
    }
    for (auto e : ev)
      if (e) keep(hipEventDestroy(e));
    ev.clear();
    dst.clear();
    pairs.clear();
    const hipError_t r = err;
    err = hipSuccess;
    return r;
  }
};
}  // namespace

// real float64 flops of a batch of complex products C = C0 + alpha (A B + A2 B2):
// 8 m n k per product
static double gemm_flops(const std::vector<GemmDesc>& v) {
  double f = 0.0;
  for (const GemmDesc& G : v) f += 8.0 * G.m * G.n * (double)(G.k + G.k2);
  return f;
}

static int row_width(const mlh_stack_s* s, int i) {
  // columns of the level-0 row block [A'_ii | A'_{i,i-1} | A'_{i,i+1} | f~_i]
  return s->n[i] + (i > 0 ? s->n[i - 1] : 0) + (i + 1 < s->I ? s->n[i + 1] : 0) + 1;
}

// how one solve call runs and where its outputs go
struct SolveOpts {
  int stop_phase = 0;            // inspection: stop after this phase (0 = whole solve)
  mlh_profile* prof = nullptr;   // time every launch (one stream, no graph)
  bool on_device = false;        // outputs are device pointers; no host wait
  bool noalloc = false;          // workspace in the context's fixed scratch; no allocation, no graph
  unsigned long long* tstamp = nullptr;  // device [1 + n_angles]: clock at the start, then per angle at its end
  bool keep_views = false;       // leave the first system's workspace views in the inspected stack
  // adjoint: after the Schur complements, solve the transposed block system
  // A'^T z = w, w_1 = the row of X_1 that gives each angle's zeroth reflected
  // amplitude (adj_q0[a]: its index in the angle's order window); z is
  // returned as the densities; no Bragg extraction
  bool adjoint = false;
  const std::vector<int>* adj_q0 = nullptr;
  struct SysViews* views = nullptr;  // per system: the workspace left by the solve (one batch only)
};

// the workspace of one system after a solve: least-squares solutions X_j
// (ld ldX[j]) and factors S_j, T_j per layer, densities eta_i per interface
struct SysViews {
  std::vector<std::vector<cplx*>> X, S, Th, eta;
  std::vector<std::vector<int>> ldX;
};

// one system of a solve: the angles of one stack whose Bloch phases alpha
// agree (kappa_0 on one grid of spacing 2 pi/d, Sec. 3.4); they share every
// matrix and take one right-hand-side column each
struct SysSpec {
  mlh_stack_s* s;
  std::vector<int> ang;  // indices into the call's angle list
};

// where one angle's results go (host or device memory, per SolveOpts)
struct AngleOut {
  double* aU;       // 2K+1 complex
  double* aD;
  int32_t* orders;  // 2K+1 labels, may be null
  double* flux;     // may be null
  double* eta;      // N_den complex, may be null
};

static void group_by_alpha(mlh_stack_s* s, int n_angles, const double* theta, int first, std::vector<SysSpec>& out) {
  std::vector<double> tfrac;
  const size_t base = out.size();
  for (int a = 0; a < n_angles; ++a) {
    const double t = s->d * s->k[0] * std::cos(theta[first + a]) / (2.0 * kPi);
    const double f = t - std::floor(t);
    int g = -1;
    for (size_t q = 0; q < tfrac.size() && g < 0; ++q) {
      const double dd = std::fabs(f - tfrac[q]);
      if (std::min(dd, 1.0 - dd) < kAlphaTol) g = (int)q;
    }
    if (g < 0) {
      out.push_back(SysSpec{s, {}});
      tfrac.push_back(f);
      g = (int)tfrac.size() - 1;
    }
    out[base + g].ang.push_back(first + a);
  }
}

// Solve the systems `sys` (of one or several stacks) in batches that share
// every launch.  theta[a] and outs[a] belong to angle a of the call;
// h_flux[a] receives each angle's flux error on the host unless the outputs
// are on the device and no accuracy check asked for them (flux_to_host).
static mlh_status solve_systems(Runner& RN, mlh_ctx ctx, const mlh_tuning& tune, const std::vector<SysSpec>& sys,
                                const double* theta, const std::vector<AngleOut>& outs, const SolveOpts& opt,
                                bool flux_to_host, std::vector<double>& h_flux, mlh_stack_s* inspect) {
  const int stop_phase = opt.stop_phase;
  mlh_profile* const prof = opt.prof;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int NS = (int)sys.size();
  bool want_eta = false;
  for (const AngleOut& o : outs) want_eta = want_eta || o.eta;
  const bool eta_stage = want_eta && !opt.on_device;  // host densities go through a device row per angle
  // ---- per-stack shapes
  struct Shape {
    const mlh_stack_s* s;
    int I = 0, maxn = 0;
    std::vector<int> nL0, nU0;
    std::vector<int64_t> den_off;  // offset of eta_i in a row of N_den densities
  };
  std::vector<Shape> shp;
  std::vector<int> sidx(NS);
  for (int b = 0; b < NS; ++b) {
    int q = -1;
    for (size_t t = 0; t < shp.size() && q < 0; ++t)
      if (shp[t].s == sys[b].s) q = (int)t;
    if (q < 0) {
      Shape sh;
      const mlh_stack_s* s = sys[b].s;
      sh.s = s;
      sh.I = s->I;
      sh.nL0.resize(s->I);
      sh.nU0.resize(s->I);
      sh.den_off.assign(s->I + 1, 0);
      for (int i = 0; i < s->I; ++i) {
        sh.maxn = std::max(sh.maxn, s->n[i]);
        sh.nL0[i] = i > 0 ? s->n[i - 1] : 0;
        sh.nU0[i] = i + 1 < s->I ? s->n[i + 1] : 0;
        sh.den_off[i + 1] = sh.den_off[i] + s->n[i];
      }
      shp.push_back(std::move(sh));
      q = (int)shp.size() - 1;
    }
    sidx[b] = q;
  }
  // ---- workspace of one system: two row-block buffers per interface (the
  //      reduction reads one and writes the other), least-squares systems,
  //      eta (one column per angle), Gauss-Jordan scratch per interface,
  //      outputs per angle
  auto plan = [&](int b, Arena& A, std::vector<size_t>* offs) {
    const mlh_stack_s* s = sys[b].s;
    const Shape& sh = shp[sidx[b]];
    const int I = sh.I, rb = (int)sys[b].ang.size();
    const std::vector<int>& n = s->n;
    auto R = [&](size_t bytes) {
      const size_t o = A.reserve(bytes);
      if (offs) offs->push_back(o);
    };
    for (int w = 0; w < 2; ++w)
      for (int i = 0; i < I; ++i) R(cbytes((size_t)n[i] * (n[i] + 2 * sh.maxn + rb)));
    for (int j = 0; j <= I; ++j) {
      int m, c, nc;
      layer_dims(s, j, m, c, nc);
      R(cbytes((size_t)(m + c) * (c + nc)));  // [S | RHS]
      R(cbytes((size_t)((c + kHqNb - 1) / kHqNb) * kHqNb * kHqNb));
    }
    for (int i = 0; i < I; ++i) R(cbytes((size_t)n[i] * rb));
    for (int i = 0; i < I; ++i) {
      const size_t steps = (size_t)(n[i] + kGjeNb - 1) / kGjeNb;
      R(cbytes(steps * kGjeNb * kGjeNb));
      R(sizeof(int) * steps * kGjePivStride);
    }
    R(cbytes((size_t)2 * s->nK * rb));
    R(sizeof(double) * rb);
    R(sizeof(int) * s->nK * rb);
    if (eta_stage) R(cbytes((size_t)sh.den_off[I] * rb));
  };
  std::vector<size_t> per(NS), dper(NS);
  for (int b = 0; b < NS; ++b) {
    Arena A;
    plan(b, A, nullptr);
    per[b] = (A.off + 255) & ~size_t(255);
    const size_t I = (size_t)shp[sidx[b]].I, rb = sys[b].ang.size();
    dper[b] = sizeof(AsmJob) * (10 * (I + 2)) + sizeof(GemmDesc) * (8 * I + 8) + sizeof(HqDesc) * (I + 1) +
              sizeof(GjeDesc) * (I + 1) + sizeof(GemvDesc) * (I + 1) + sizeof(AngleDesc) * rb + sizeof(EtaSeg) * I +
              sizeof(EtaDst) * rb + sizeof(TransposeJob) * (4 * I + rb + 4);
  }
  // alignment slack of one batch's descriptor uploads (3 lists per level)
  const size_t slack = (size_t)256 * (3 * 64 + 24) + 4096;
  // ---- batches of consecutive systems: as many as the memory holds, and at
  //      most 65535 matrices per launch (one per grid row)
  size_t budget;
  if (opt.noalloc) {
    budget = kScratchBytes - slack;
  } else {
    size_t freeb = 0, totb = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &totb));
    budget = (size_t)(0.8 * (double)(freeb + RN.wbytes));
    budget = budget > slack ? budget - slack : 0;
    // a caller's cap on the workspace (batches shrink to fit; a batch
    // always holds at least one system)
    if (const char* lim = std::getenv("MLH_WORKSPACE_LIMIT_MB")) {
      const double mb = std::atof(lim);
      if (mb > 0) budget = std::min(budget, (size_t)(mb * 1048576.0));
    }
  }
  std::vector<int> bstart = {0};
  size_t need = 0;
  {
    size_t acc = 0;
    int64_t rows = 0;
    for (int b = 0; b < NS; ++b) {
      const size_t sz = per[b] + dper[b];
      const int64_t r = shp[sidx[b]].I + 1;
      if (b > bstart.back() && (acc + sz > budget || rows + r > 65535)) {
        bstart.push_back(b);
        acc = 0;
        rows = 0;
      }
      acc += sz;
      rows += r;
      need = std::max(need, acc);
    }
    bstart.push_back(NS);
    need += slack;
  }
  if (opt.views && bstart.size() > 2)
    return fail(MLH_E_UNSUPPORTED, "the adjoint needs every system of the call in one batch: fewer angles per call");
  char* wbase = nullptr;
  if (opt.noalloc) {
    if (need > kScratchBytes) {
      char msg[200];
      std::snprintf(msg, sizeof msg,
                    "one system of this solve needs %.1f MiB of workspace; the allocation-free solve holds at "
                    "most %.1f MiB", need / 1048576.0, kScratchBytes / 1048576.0);
      return fail(MLH_E_UNSUPPORTED, msg);
    }
    wbase = ctx->scratch;
  } else {
    if (need > RN.wbytes) {
      if (RN.gexec) {
        const hipError_t de = hipGraphExecDestroy(RN.gexec);
        RN.gexec = nullptr;
        HIP_TRY(de);
      }
      if (RN.wmem) HIP_TRY(hipFree(RN.wmem));
      RN.wmem = nullptr;
      RN.wbytes = 0;
      hipError_t e = hipMalloc((void**)&RN.wmem, need);
      if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE, "solve workspace");
      RN.wbytes = need;
    }
    wbase = RN.wmem;
  }
  if (RN.num_cu == 0) HIP_TRY(hipDeviceGetAttribute(&RN.num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  h_flux.assign(outs.size(), 0.0);
  for (size_t bi = 0; bi + 1 < bstart.size(); ++bi) {
    const int b0 = bstart[bi], nb = bstart[bi + 1] - b0;
    auto SY = [&](int b) -> const SysSpec& { return sys[b0 + b]; };
    auto SH = [&](int b) -> const Shape& { return shp[sidx[b0 + b]]; };
    auto R_of = [&](int b) { return (int)SY(b).ang.size(); };
    int nang = 0, rchunk = 1;
    std::vector<size_t> sys_off(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      nang += R_of(b);
      rchunk = std::max(rchunk, R_of(b));
      sys_off[b + 1] = sys_off[b] + per[b0 + b];
    }
    char* dbase = wbase + sys_off[nb];
    struct View {
      std::vector<cplx*> W[2], S, Th, RHS, eta, M1;
      std::vector<int*> piv;
      cplx* out;  // per angle: a^U (nK) then a^D (nK)
      double* flux;
      int* orders;
      cplx* eta_rows = nullptr;  // host densities: one row of N_den per angle
    };
    std::vector<View> V(nb);
    for (int b = 0; b < nb; ++b) {
      std::vector<size_t> offs;
      {
        Arena A;
        plan(b0 + b, A, &offs);
      }
      char* wb = wbase + sys_off[b];
      size_t k = 0;
      auto C = [&]() { return reinterpret_cast<cplx*>(wb + offs[k++]); };
      View& v = V[b];
      const int I = SH(b).I;
      for (int i = 0; i < I; ++i) v.W[0].push_back(C());
      for (int i = 0; i < I; ++i) v.W[1].push_back(C());
      for (int j = 0; j <= I; ++j) {
        int m, c, nc;
        layer_dims(SY(b).s, j, m, c, nc);
        cplx* aug = C();
        v.S.push_back(aug);
        v.RHS.push_back(aug + (size_t)(m + c) * c);
        v.Th.push_back(C());
      }
      for (int i = 0; i < I; ++i) v.eta.push_back(C());
      for (int i = 0; i < I; ++i) {
        v.M1.push_back(C());
        v.piv.push_back(reinterpret_cast<int*>(wb + offs[k++]));
      }
      v.out = C();
      v.flux = reinterpret_cast<double*>(wb + offs[k++]);
      v.orders = reinterpret_cast<int*>(wb + offs[k++]);
      if (eta_stage) v.eta_rows = C();
    }
    auto Dblk = [&](int b, int i) { return V[b].W[0][i]; };
    auto Lblk = [&](int b, int i) { return V[b].W[0][i] + (size_t)SY(b).s->n[i] * SY(b).s->n[i]; };
    auto Ublk = [&](int b, int i) {
      const std::vector<int>& n = SY(b).s->n;
      return V[b].W[0][i] + (size_t)n[i] * (n[i] + SH(b).nL0[i]);
    };
    auto Fcol = [&](int b, int i) {
      const std::vector<int>& n = SY(b).s->n;
      return V[b].W[0][i] + (size_t)n[i] * (n[i] + SH(b).nL0[i] + SH(b).nU0[i]);
    };
    // ---- descriptors
    // two job lists: the least-squares inputs, which the layer solves wait
    // for, and the blocks of the block-tridiagonal system, which only the
    // Schur updates read (so they assemble inside the panel launches of the
    // layer solves, on the compute units those leave idle)
    struct AsmList {
      std::vector<AsmJob> jobs;
      int64_t tiles = 0;
    } asm_ls, asm_blk;
    auto asm_add = [&](AsmList& L, cplx* dst, int ldd, int rows, int cols, int np, const cplx* const* src, int lds,
                       const cplx* coef) {
      if (rows <= 0 || cols <= 0) return;
      AsmJob J{};
      J.dst = dst;
      J.ldd = ldd;
      J.rows = rows;
      J.cols = cols;
      J.npieces = np;
      J.lds = lds;
      for (int p = 0; p < np; ++p) {
        J.src[p] = src[p];
        J.coef[p] = coef[p];
      }
      J.tile_begin = (int)L.tiles;
      L.tiles += ((int64_t)rows * cols + kAsmTile - 1) / kAsmTile;
      L.jobs.push_back(J);
    };
    // C = C0 + alpha (A B + A2 B2); m x nn output, inner sizes k and k2
    auto gemm_add = [&](std::vector<GemmDesc>& vec, int& tiles, cplx* Cm, int ldc, const cplx* C0, int ldc0, int m,
                        int nn, const cplx* A, int lda, const cplx* Bm, int ldb, int k, const cplx* A2, int lda2,
                        const cplx* B2, int ldb2, int k2) {
      if (m <= 0 || nn <= 0) return;
      GemmDesc G{};
      G.A = A;
      G.B = Bm;
      G.k = k;
      G.lda = lda;
      G.ldb = ldb;
      G.A2 = A2;
      G.B2 = B2;
      G.k2 = k2;
      G.lda2 = lda2;
      G.ldb2 = ldb2;
      G.C = Cm;
      G.ldc = ldc;
      G.C0 = C0;
      G.ldc0 = ldc0;
      G.alpha = cx(-1.0, 0.0);
      G.m = m;
      G.n = nn;
      G.tiles_m = (m + kGemmTile - 1) / kGemmTile;
      G.tile_begin = tiles;
      tiles += G.tiles_m * ((nn + kGemmTile - 1) / kGemmTile);
      vec.push_back(G);
    };
    std::vector<GemmDesc> gs;
    int gtiles = 0;
    std::vector<HqDesc> hq;
    int maxc = 0, maxcols = 0, maxncol = 0;
    struct HqClass {
      int n = 0, maxc = 0, maxncol = 0, maxrows = 0;
    } hq_small, hq_large;
    std::vector<AngleDesc> angs;
    const cplx one = cx(1, 0);
    for (int b = 0; b < nb; ++b) {
      View& v = V[b];
      const mlh_stack_s* s = SY(b).s;
      const int I = s->I, P = s->P, nK = s->nK;
      const std::vector<int>& n = s->n;
      const int rb = R_of(b);
      const double th = theta[SY(b).ang[0]];
      const double ph = s->d * s->k[0] * std::cos(th);  // alpha = e^{i ph}, eq. (2)
      const cplx a_m1 = cpow_alpha(ph, -1), a_p1 = cpow_alpha(ph, 1), a_m2 = cpow_alpha(ph, -2);
      const cplx c3[3] = {a_m1, one, a_p1};
      const cplx cC[2] = {a_m2, cx(-a_p1.re, -a_p1.im)};
      const cplx cQ[2] = {a_m1, cx(-1, 0)};
      for (int i = 0; i < I; ++i) {
        const size_t pe = (size_t)n[i] * n[i];
        const cplx* src[3] = {s->A_self[i], s->A_self[i] + pe, s->A_self[i] + 2 * pe};
        asm_add(asm_blk, Dblk(b, i), n[i], n[i], n[i], 3, src, n[i], c3);
        if (i > 0) asm_add(asm_blk, Fcol(b, i), n[i], n[i], rb, 0, src, n[i], c3);  // f_i = 0 below Gamma_1
        if (i + 1 < I) {
          const size_t pu = (size_t)n[i] * n[i + 1];
          const cplx* su[3] = {s->A_up[i], s->A_up[i] + pu, s->A_up[i] + 2 * pu};
          asm_add(asm_blk, Ublk(b, i), n[i], n[i], n[i + 1], 3, su, n[i], c3);
          const cplx* sd[3] = {s->A_dn[i], s->A_dn[i] + pu, s->A_dn[i] + 2 * pu};
          asm_add(asm_blk, Lblk(b, i + 1), n[i + 1], n[i + 1], n[i], 3, sd, n[i + 1], c3);
        }
      }
      for (int j = 0; j <= I; ++j) {
        int m, c, nc;
        layer_dims(s, j, m, c, nc);
        const int M = m + c;
        const int mw2 = 2 * s->Mw, mud2 = 2 * s->Mud;
        const size_t qe = (size_t)mw2 * P;
        const cplx* sq[2] = {s->Q[j], s->Q[j] + qe};
        asm_add(asm_ls, v.S[j], M, mw2, P, 2, sq, mw2, cQ);
        if (j == 0 || j == I) {
          const cplx* vv[1] = {j == 0 ? s->V_U : s->V_D};
          asm_add(asm_ls, v.S[j] + mw2, M, mud2, P, 1, vv, mud2, &one);
          asm_add(asm_ls, v.S[j] + (size_t)P * M, M, mw2, nK, 0, vv, mud2, &one);
          const int ci = j == 0 ? 0 : I - 1;
          const size_t ce = (size_t)mw2 * n[ci];
          const cplx* cs = j == 0 ? s->C_own[0] : s->C_above[I];
          const cplx* sc[2] = {cs, cs + ce};
          asm_add(asm_ls, v.RHS[j], M, mw2, n[ci], 2, sc, mw2, cC);
          const size_t ze = (size_t)mud2 * n[ci];
          const cplx* zb = j == 0 ? s->Z_U : s->Z_D;
          const cplx* sz[3] = {zb, zb + ze, zb + 2 * ze};
          asm_add(asm_ls, v.RHS[j] + mw2, M, mud2, n[ci], 3, sz, mud2, c3);
          asm_add(asm_ls, v.RHS[j] + m, M, c, n[ci], 0, sz, mud2, c3);
        } else {
          const size_t ea = (size_t)mw2 * n[j - 1], eo = (size_t)mw2 * n[j];
          const cplx* sa[2] = {s->C_above[j], s->C_above[j] + ea};
          const cplx* so[2] = {s->C_own[j], s->C_own[j] + eo};
          asm_add(asm_ls, v.RHS[j], M, mw2, n[j - 1], 2, sa, mw2, cC);
          asm_add(asm_ls, v.RHS[j] + (size_t)n[j - 1] * M, M, mw2, n[j], 2, so, mw2, cC);
          asm_add(asm_ls, v.RHS[j] + m, M, c, nc, 0, sa, mw2, cC);
        }
        HqDesc H{};
        H.A = v.S[j];
        H.T = v.Th[j];
        H.mu_rel = s->mu;
        H.m = m;
        H.c = c;
        H.ncol = nc;
        hq.push_back(H);
        maxc = std::max(maxc, c);
        maxcols = std::max(maxcols, c + nc);
        maxncol = std::max(maxncol, nc);
      }
      // Schur complements eq. (74)-(78): A' = A - B X, in place; each
      // descriptor owns its output block
      for (int i = 0; i < I; ++i) {
        int m0, c0, nc0, m1, c1, nc1;
        layer_dims(s, i, m0, c0, nc0);
        layer_dims(s, i + 1, m1, c1, nc1);
        const int Ma = m0 + c0, Mb = m1 + c1;
        const cplx* Xa = (i == 0) ? v.RHS[0] : v.RHS[i] + (size_t)n[i - 1] * Ma;
        const cplx* Xb = v.RHS[i + 1];
        gemm_add(gs, gtiles, Dblk(b, i), n[i], Dblk(b, i), n[i], n[i], n[i], s->B_own[i], n[i], Xa, Ma, P,
                 s->B_below[i], n[i], Xb, Mb, P);
        if (i + 1 < I)
          gemm_add(gs, gtiles, Ublk(b, i), n[i], Ublk(b, i), n[i], n[i], n[i + 1], s->B_below[i], n[i],
                   v.RHS[i + 1] + (size_t)n[i] * Mb, Mb, P, nullptr, 1, nullptr, 1, 0);
        if (i > 0)
          gemm_add(gs, gtiles, Lblk(b, i), n[i], Lblk(b, i), n[i], n[i], n[i - 1], s->B_own[i], n[i], v.RHS[i], Ma, P,
                   nullptr, 1, nullptr, 1, 0);
      }
      int m0, c0, nc0, mI, cI, ncI;
      layer_dims(s, 0, m0, c0, nc0);
      layer_dims(s, I, mI, cI, ncI);
      StackConsts sc{};
      sc.x1 = s->gx[0];
      sc.y1 = s->gy[0];
      sc.nx1 = s->gnx[0];
      sc.ny1 = s->gny[0];
      sc.xud = s->ud_x;
      sc.y0_1 = s->curves[0].y0;
      sc.d = s->d;
      sc.k1 = s->k[0];
      sc.kI1 = s->k[I];
      sc.N1 = s->N[0];
      sc.NI = s->N[I - 1];
      sc.Mw = s->Mw;
      sc.Mud = s->Mud;
      sc.P = P;
      sc.K = s->K;
      for (int q = 0; q < rb; ++q) {  // one descriptor per angle of the system
        AngleDesc A{};
        A.sc = sc;
        A.theta = theta[SY(b).ang[q]];
        A.owner = q == 0;
        A.S0 = v.S[0];
        A.ldS0 = m0 + c0;
        A.SI = v.S[I];
        A.ldSI = mI + cI;
        A.F0 = Fcol(b, 0) + (size_t)q * n[0];
        A.X0 = v.RHS[0];
        A.ldX0 = m0 + c0;
        A.XI = v.RHS[I];
        A.ldXI = mI + cI;
        A.eta0 = v.eta[0] + (size_t)q * n[0];
        A.etaI = v.eta[I - 1] + (size_t)q * n[I - 1];
        A.aU = v.out + (size_t)2 * nK * q;
        A.aD = A.aU + nK;
        A.orders = v.orders + (size_t)nK * q;
        A.flux = v.flux + q;
        A.tdone = opt.tstamp ? opt.tstamp + 1 + SY(b).ang[q] : nullptr;
        angs.push_back(A);
      }
    }
    // adjoint: the transposed block system in the second row-block buffer,
    // [D_i^T | U_{i-1}^T | L_{i+1}^T | w_i], which the reduction then reads
    // first (A'^T has (A'^T)_{i,i-1} = A'_{i-1,i}^T and (A'^T)_{i,i+1} =
    // A'_{i+1,i}^T, of the same shapes as L_i and U_i)
    std::vector<TransposeJob> tjobs;
    int ttiles = 0;
    auto tadd = [&](const cplx* src, int lds, cplx* dst, int ldd, int rows, int cols) {
      if (rows <= 0 || cols <= 0) return;
      TransposeJob T{};
      T.src = src;
      T.lds = lds;
      T.dst = dst;
      T.ldd = ldd;
      T.rows = rows;
      T.cols = cols;
      T.tile_begin = ttiles;
      ttiles += ((rows + 31) / 32) * ((cols + 31) / 32);
      tjobs.push_back(T);
    };
    if (opt.adjoint) {
      for (int b = 0; b < nb; ++b) {
        const mlh_stack_s* s = SY(b).s;
        const std::vector<int>& n = s->n;
        const Shape& sh = SH(b);
        for (int i = 0; i < sh.I; ++i) {
          cplx* W1 = V[b].W[1][i];
          tadd(Dblk(b, i), n[i], W1, n[i], n[i], n[i]);
          if (i > 0) tadd(Ublk(b, i - 1), n[i - 1], W1 + (size_t)n[i] * n[i], n[i], n[i], n[i - 1]);
          if (i + 1 < sh.I)
            tadd(Lblk(b, i + 1), n[i + 1], W1 + (size_t)n[i] * (n[i] + sh.nL0[i]), n[i], n[i], n[i + 1]);
          cplx* F1 = W1 + (size_t)n[i] * (n[i] + sh.nL0[i] + sh.nU0[i]);
          int m0, c0, nc0;
          layer_dims(s, 0, m0, c0, nc0);
          for (int q = 0; q < R_of(b); ++q) {
            if (i == 0) {  // the a0 row of X_1, as a column
              const int q0 = (*opt.adj_q0)[SY(b).ang[q]];
              tadd(V[b].RHS[0] + s->P + q0, m0 + c0, F1 + (size_t)q * n[0], n[0], n[0], 1);
            } else {
              tadd(nullptr, 1, F1 + (size_t)q * n[i], n[i], n[i], 1);
            }
          }
        }
      }
    }
    // layers with at most kHqRhsSmallRows rows first: the right-hand-side
    // kernel is launched once per size class (the other kernels take each
    // descriptor on its own)
    std::stable_partition(hq.begin(), hq.end(), [](const HqDesc& H) { return H.m + H.c <= kHqRhsSmallRows; });
    for (const HqDesc& H : hq) {
      HqClass& g = H.m + H.c <= kHqRhsSmallRows ? hq_small : hq_large;
      ++g.n;
      g.maxc = std::max(g.maxc, H.c);
      g.maxncol = std::max(g.maxncol, H.ncol);
      g.maxrows = std::max(g.maxrows, H.m + H.c);
    }
    // ---- block-tridiagonal solve by cyclic reduction (the paper's block LU,
    //      Sec. 3.3, reordered so that every level eliminates half of the
    //      remaining blocks at once).  Block j holds [D_j | L_j | U_j | f_j]
    //      with L_j / U_j its couplings to the left / right neighbour in the
    //      active set.  Eliminating e: [XL | XU | xf] = D_e^{-1} [L_e | U_e | f_e];
    //      a kept neighbour j then becomes
    //        D_j - L_j XU_{e_l} - U_j XL_{e_r},  f_j - L_j xf_{e_l} - U_j xf_{e_r},
    //        L_j' = -L_j XL_{e_l},  U_j' = -U_j XU_{e_r}.
    //      Each stack of the batch has its own sequence of levels; level l of
    //      every stack shares the launches of level l.
    struct Level {
      std::vector<GjeDesc> gje;  // orders <= kRhsMaxN16 first (size classes of the right-hand-side kernel)
      int maxn = 0, maxcol = 0, maxrhs = 0;
      int nsmall = 0, rhs_small = 0, rhs_large = 0;
      bool rhs_in_step = false;  // right-hand sides eliminated with the matrix, no replay
      std::vector<GemmDesc> upd;
      int upd_tiles = 0;
      std::vector<GemvDesc> back;
      int backn = 0;
    };
    std::vector<Level> levels;
    auto Wp = [&](int b, int i, int which) { return V[b].W[which][i]; };
    auto merge_level = [&](size_t l, Level& lv) {
      if (levels.size() <= l) levels.resize(l + 1);
      Level& M = levels[l];
      for (GemmDesc G : lv.upd) {
        G.tile_begin += M.upd_tiles;
        M.upd.push_back(G);
      }
      M.upd_tiles += lv.upd_tiles;
      M.gje.insert(M.gje.end(), lv.gje.begin(), lv.gje.end());
      M.back.insert(M.back.end(), lv.back.begin(), lv.back.end());
      M.maxn = std::max(M.maxn, lv.maxn);
      M.maxcol = std::max(M.maxcol, lv.maxcol);
      M.maxrhs = std::max(M.maxrhs, lv.maxrhs);
      M.backn = std::max(M.backn, lv.backn);
    };
    for (size_t t = 0; t < shp.size(); ++t) {
      std::vector<int> bs;  // systems of this batch on stack t
      for (int b = 0; b < nb; ++b)
        if (sidx[b0 + b] == (int)t) bs.push_back(b);
      if (bs.empty()) continue;
      const Shape& sh = shp[t];
      const int I = sh.I;
      const std::vector<int>& n = sh.s->n;
      std::vector<int> cur(I, opt.adjoint ? 1 : 0), nLc(sh.nL0), nUc(sh.nU0);
      std::vector<int> S_act(I);
      for (int i = 0; i < I; ++i) S_act[i] = i;
      for (size_t lidx = 0;; ++lidx) {
        Level lv;
        const int m = (int)S_act.size();
        if (m == 1) {
          const int j = S_act[0];
          for (int b : bs) {
            GjeDesc G{};
            G.W = Wp(b, j, cur[j]);
            G.M1 = V[b].M1[j];
            G.piv = V[b].piv[j];
            G.n = n[j];
            G.ncol = n[j] + nLc[j] + nUc[j] + R_of(b);
            lv.gje.push_back(G);
            lv.maxcol = std::max(lv.maxcol, G.ncol);
            lv.maxrhs = std::max(lv.maxrhs, G.ncol - G.n);
            GemvDesc Gv{};
            Gv.g = G.W + (size_t)n[j] * (n[j] + nLc[j] + nUc[j]);
            Gv.y = V[b].eta[j];
            Gv.n = n[j];
            Gv.r = R_of(b);
            lv.back.push_back(Gv);
          }
          lv.maxn = n[j];
          lv.backn = n[j];
          merge_level(lidx, lv);
          break;
        }
        // eliminate odd positions
        for (int p = 1; p < m; p += 2) {
          const int e = S_act[p], left = S_act[p - 1], right = (p + 1 < m) ? S_act[p + 1] : -1;
          for (int b : bs) {
            GjeDesc G{};
            G.W = Wp(b, e, cur[e]);
            G.M1 = V[b].M1[e];
            G.piv = V[b].piv[e];
            G.n = n[e];
            G.ncol = n[e] + nLc[e] + nUc[e] + R_of(b);
            lv.gje.push_back(G);
            lv.maxcol = std::max(lv.maxcol, G.ncol);
            lv.maxrhs = std::max(lv.maxrhs, G.ncol - G.n);
            const cplx* X = G.W + (size_t)n[e] * n[e];
            GemvDesc Gv{};
            Gv.U1 = X;
            Gv.m1 = nLc[e];
            Gv.x1 = V[b].eta[left];
            Gv.U2 = X + (size_t)n[e] * nLc[e];
            Gv.m2 = right >= 0 ? nUc[e] : 0;
            Gv.x2 = right >= 0 ? V[b].eta[right] : nullptr;
            Gv.g = X + (size_t)n[e] * (nLc[e] + nUc[e]);
            Gv.y = V[b].eta[e];
            Gv.n = n[e];
            Gv.r = R_of(b);
            lv.back.push_back(Gv);
          }
          lv.maxn = std::max(lv.maxn, n[e]);
          lv.backn = std::max(lv.backn, n[e]);
        }
        // update the kept blocks
        std::vector<int> newL(I), newU(I);
        for (int p = 0; p < m; p += 2) {
          const int j = S_act[p];
          const int el = p >= 1 ? S_act[p - 1] : -1, er = p + 1 < m ? S_act[p + 1] : -1;
          const int ll = p >= 2 ? S_act[p - 2] : -1, rr = p + 2 < m ? S_act[p + 2] : -1;
          const int nLn = ll >= 0 ? n[ll] : 0, nUn = rr >= 0 ? n[rr] : 0;
          newL[j] = nLn;
          newU[j] = nUn;
          const int nj = n[j];
          for (int b : bs) {
            cplx* Wc = Wp(b, j, cur[j]);
            cplx* Wn = Wp(b, j, cur[j] ^ 1);
            const cplx* Lj = Wc + (size_t)nj * nj;
            const cplx* Uj = Wc + (size_t)nj * (nj + nLc[j]);
            const cplx* fj = Wc + (size_t)nj * (nj + nLc[j] + nUc[j]);
            const cplx *XLl = nullptr, *XUl = nullptr, *xfl = nullptr, *XLr = nullptr, *XUr = nullptr, *xfr = nullptr;
            int nel = 0, ner = 0;
            if (el >= 0) {
              nel = n[el];
              const cplx* X = Wp(b, el, cur[el]) + (size_t)nel * nel;
              XLl = X;
              XUl = X + (size_t)nel * nLc[el];
              xfl = X + (size_t)nel * (nLc[el] + nUc[el]);
            }
            if (er >= 0) {
              ner = n[er];
              const cplx* X = Wp(b, er, cur[er]) + (size_t)ner * ner;
              XLr = X;
              XUr = X + (size_t)ner * nLc[er];
              xfr = X + (size_t)ner * (nLc[er] + nUc[er]);
            }
            // D and f (one or two products each)
            if (el >= 0 && er >= 0) {
              gemm_add(lv.upd, lv.upd_tiles, Wn, nj, Wc, nj, nj, nj, Lj, nj, XUl, nel, nel, Uj, nj, XLr, ner, ner);
              gemm_add(lv.upd, lv.upd_tiles, Wn + (size_t)nj * (nj + nLn + nUn), nj, fj, nj, nj, R_of(b), Lj, nj, xfl,
                       nel, nel, Uj, nj, xfr, ner, ner);
            } else if (el >= 0) {
              gemm_add(lv.upd, lv.upd_tiles, Wn, nj, Wc, nj, nj, nj, Lj, nj, XUl, nel, nel, nullptr, 1, nullptr, 1, 0);
              gemm_add(lv.upd, lv.upd_tiles, Wn + (size_t)nj * (nj + nLn + nUn), nj, fj, nj, nj, R_of(b), Lj, nj, xfl,
                       nel, nel, nullptr, 1, nullptr, 1, 0);
            } else {
              gemm_add(lv.upd, lv.upd_tiles, Wn, nj, Wc, nj, nj, nj, Uj, nj, XLr, ner, ner, nullptr, 1, nullptr, 1, 0);
              gemm_add(lv.upd, lv.upd_tiles, Wn + (size_t)nj * (nj + nLn + nUn), nj, fj, nj, nj, R_of(b), Uj, nj, xfr,
                       ner, ner, nullptr, 1, nullptr, 1, 0);
            }
            if (ll >= 0)
              gemm_add(lv.upd, lv.upd_tiles, Wn + (size_t)nj * nj, nj, nullptr, nj, nj, nLn, Lj, nj, XLl, nel, nel,
                       nullptr, 1, nullptr, 1, 0);
            if (rr >= 0)
              gemm_add(lv.upd, lv.upd_tiles, Wn + (size_t)nj * (nj + nLn), nj, nullptr, nj, nj, nUn, Uj, nj, XUr, ner,
                       ner, nullptr, 1, nullptr, 1, 0);
          }
        }
        merge_level(lidx, lv);
        std::vector<int> K;
        for (int p = 0; p < m; p += 2) {
          const int j = S_act[p];
          cur[j] ^= 1;
          nLc[j] = newL[j];
          nUc[j] = newU[j];
          K.push_back(j);
        }
        S_act = K;
      }
    }
    for (Level& lv : levels) {
      std::stable_partition(lv.gje.begin(), lv.gje.end(), [](const GjeDesc& G) { return G.n <= kRhsMaxN16; });
      for (const GjeDesc& G : lv.gje) {
        if (G.n <= kRhsMaxN16) {
          ++lv.nsmall;
          lv.rhs_small = std::max(lv.rhs_small, G.ncol - G.n);
        } else {
          lv.rhs_large = std::max(lv.rhs_large, G.ncol - G.n);
        }
      }
    }
    // Levels with few matrices: the compute units idle beside the panels,
    // whose chain sets the pace, so the update workgroups of each step take
    // the right-hand-side columns as well (Gauss-Jordan on [D | B]) in place
    // of the replay after the last step, when a step launch needs at most a
    // few workgroups per compute unit (a workgroup fills a unit; the bound
    // is a launch choice, 300 per 100 units unless tuned).
    for (Level& lv : levels)
      lv.rhs_in_step =
          gje_step_fits(lv.maxn) && (int64_t)gje_step_max_blocks((int)lv.gje.size(), lv.maxn, lv.maxcol, lv.maxrhs) *
                                            100 <= (int64_t)RN.num_cu * tune.rhs_in_step_pct;
    // ---- upload descriptors
    size_t doff = 0;
    std::vector<char> hdesc;
    auto push = [&](const void* p, size_t bytes) {
      const size_t o = (doff + 255) & ~size_t(255);
      hdesc.resize(o + bytes);
      if (bytes && p) std::memcpy(hdesc.data() + o, p, bytes);
      doff = o + bytes;
      return o;
    };
    const size_t oi = push(nullptr, sizeof(int) * 4);
    std::memset(hdesc.data() + oi, 0, sizeof(int) * 4);
    int* d_info = reinterpret_cast<int*>(dbase + oi);
    for (auto& lv : levels)
      for (auto& G : lv.gje) G.info = d_info;
    const size_t o_asm_ls = push(asm_ls.jobs.data(), sizeof(AsmJob) * asm_ls.jobs.size());
    const size_t o_asm_blk = push(asm_blk.jobs.data(), sizeof(AsmJob) * asm_blk.jobs.size());
    const size_t o_gs = push(gs.data(), sizeof(GemmDesc) * gs.size());
    const size_t o_hq = push(hq.data(), sizeof(HqDesc) * hq.size());
    const size_t o_ang = push(angs.data(), sizeof(AngleDesc) * angs.size());
    const size_t o_tj = push(tjobs.data(), sizeof(TransposeJob) * tjobs.size());
    // densities: where eta_i sits in each system's workspace, and each
    // angle's output row
    size_t o_eseg = 0, o_edst = 0;
    int n_edst = 0, max_seg = 0, max_segn = 0;
    if (want_eta && stop_phase == 0) {
      std::vector<EtaSeg> eseg;
      std::vector<EtaDst> edst;
      for (int b = 0; b < nb; ++b) {
        const Shape& sh = SH(b);
        const int seg0 = (int)eseg.size();
        for (int i = 0; i < sh.I; ++i) {
          EtaSeg E{};
          E.src_off = (int64_t)(reinterpret_cast<char*>(V[b].eta[i]) - (wbase + sys_off[b]));
          E.dst_off = sh.den_off[i];
          E.n = sh.s->n[i];
          eseg.push_back(E);
          max_segn = std::max(max_segn, E.n);
        }
        max_seg = std::max(max_seg, sh.I);
        for (int q = 0; q < R_of(b); ++q) {
          const AngleOut& o = outs[SY(b).ang[q]];
          if (!o.eta) continue;
          EtaDst E{};
          E.sys_base = wbase + sys_off[b];
          E.col = q;
          E.seg0 = seg0;
          E.nseg = sh.I;
          E.dst = opt.on_device ? reinterpret_cast<cplx*>(o.eta) : V[b].eta_rows + (size_t)sh.den_off[sh.I] * q;
          edst.push_back(E);
        }
      }
      o_eseg = push(eseg.data(), sizeof(EtaSeg) * eseg.size());
      o_edst = push(edst.data(), sizeof(EtaDst) * edst.size());
      n_edst = (int)edst.size();
    }
    const int NL = (int)levels.size();
    std::vector<size_t> o_gje(NL), o_upd(NL), o_back(NL);
    for (int l = 0; l < NL; ++l) {
      o_gje[l] = push(levels[l].gje.data(), sizeof(GjeDesc) * levels[l].gje.size());
      o_upd[l] = push(levels[l].upd.data(), sizeof(GemmDesc) * levels[l].upd.size());
      o_back[l] = push(levels[l].back.data(), sizeof(GemvDesc) * levels[l].back.size());
    }
    if (dbase + doff > wbase + (opt.noalloc ? kScratchBytes : RN.wbytes))
      return fail(MLH_E_DEVICE, "descriptor space exhausted");
    HIP_TRY(hipMemcpyAsync(dbase, hdesc.data(), doff, hipMemcpyHostToDevice, st));
    // ---- launch sequence (captured into a graph and replayed when possible)
    if (!opt.noalloc && !RN.aux_stream) HIP_TRY(hipStreamCreateWithFlags(&RN.aux_stream, hipStreamNonBlocking));
    size_t ev_used = 0;
    auto ev_next = [&]() -> hipEvent_t {
      if (ev_used == RN.evpool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        RN.evpool.push_back(e);
      }
      return RN.evpool[ev_used++];
    };
    auto launch_all = [&](hipStream_t ls, EvTimer& T) -> mlh_status {
      ev_used = 0;
      double dummy = 0.0;
      auto tb = [&](double* acc) {
        if (prof) T.begin(acc ? acc : &dummy);
      };
      auto te = [&]() {
        if (prof) T.end();
      };
      const AsmJob* d_blk = reinterpret_cast<AsmJob*>(dbase + o_asm_blk);
      const int nblk = (int)asm_blk.jobs.size(), blk_tiles = (int)asm_blk.tiles;
      // the blocks ride in the panel launches unless those do not run or
      // every launch is timed on its own
      const bool blk_in_panels = tune.asm_in_panels && !prof && (stop_phase == 0 || stop_phase >= 2) && maxc > 0;
      if (opt.tstamp && bi == 0) launch_stamp(opt.tstamp, ls);
      tb(prof ? &prof->assemble_ms : nullptr);
      launch_assemble(reinterpret_cast<AsmJob*>(dbase + o_asm_ls), (int)asm_ls.jobs.size(), (int)asm_ls.tiles, ls);
      if (!blk_in_panels) launch_assemble(d_blk, nblk, blk_tiles, ls);
      te();
      const AngleDesc* d_ang = reinterpret_cast<AngleDesc*>(dbase + o_ang);
      tb(prof ? &prof->rb_setup_ms : nullptr);
      launch_rb_setup(d_ang, nang, ls);
      te();
      const HqDesc* d_hq = reinterpret_cast<HqDesc*>(dbase + o_hq);
      const int nhq = (int)hq.size();
      if (stop_phase == 0 || stop_phase >= 2) {
        tb(prof ? &prof->ls_panel_ms : nullptr);
        launch_hq_prep(d_hq, nhq, ls);
        te();
        const int npanels = (maxc + kHqNb - 1) / kHqNb;
        const int per = blk_in_panels ? (blk_tiles + npanels - 1) / npanels : 0;
        for (int k = 0, p = 0; k < maxc; k += kHqNb, ++p) {
          tb(prof ? &prof->ls_panel_ms : nullptr);
          const int t0 = std::min(p * per, blk_tiles), t1 = std::min(t0 + per, blk_tiles);
          launch_hq_panel(d_hq, nhq, k, ls, d_blk, nblk, t0, t1);
          te();
          tb(prof ? &prof->ls_update_ms : nullptr);
          launch_hq_update(d_hq, hq_small.n, hq_large.n, k, std::max(hq_small.maxc, hq_large.maxc), ls,
                           tune.ls_row_blocks);
          te();
        }
        tb(prof ? &prof->ls_rhs_ms : nullptr);
        launch_hq_rhs(d_hq, hq_small.n, hq_large.n, std::max(hq_small.maxncol, hq_large.maxncol),
                      std::max(hq_small.maxc, hq_large.maxc), ls, tune.ls_row_blocks);
        te();
      }
      if (stop_phase == 0 || stop_phase >= 3) {
        tb(prof ? &prof->schur_ms : nullptr);
        launch_gemm(reinterpret_cast<GemmDesc*>(dbase + o_gs), (int)gs.size(), gtiles, ls, tune.gemm_slab_k);
        te();
        if (prof) {
          prof->n_schur_gemm++;
          prof->schur_flops += gemm_flops(gs);
        }
        if (opt.adjoint) launch_transpose(reinterpret_cast<TransposeJob*>(dbase + o_tj), (int)tjobs.size(), ttiles, ls);
      }
      if (stop_phase == 0 || stop_phase >= 4) {
        for (int l = 0; l < NL; ++l) {
          const Level& lv = levels[l];
          const GjeDesc* dg = reinterpret_cast<GjeDesc*>(dbase + o_gje[l]);
          const int ng = (int)lv.gje.size();
          // Step s: the panel kernel applies step s - 1 to its own 16 columns
          // and factors them; the update kernel applies step s to the
          // columns from k + 32 on.  Panel s needs the update of step s - 2
          // only, so it runs while the update of step s - 1 is in flight on
          // the second stream.
          const int nsteps = (lv.maxn + kGjeNb - 1) / kGjeNb;
          const int rcol = lv.rhs_in_step ? lv.maxcol : 0;  // > 0: the updates take the right-hand sides
          const bool narrow = tune.gje_rhs_cols == 8;
          if (prof && gje_step_fits(lv.maxn)) {  // the graph's step launches, each timed on its own
            for (int st_i = 0; st_i < nsteps; ++st_i) {
              tb(&prof->gje_step_ms);
              launch_gje_step(dg, ng, st_i * kGjeNb, lv.maxn, ls, rcol, lv.maxrhs);
              te();
              prof->n_gje_step++;
            }
            if (lv.rhs_in_step) {
              tb(&prof->gje_update_ms);
              launch_gje_update(dg, ng, (nsteps - 1) * kGjeNb, lv.maxn, kGjeNb, 1 << 30, ls, rcol, lv.maxrhs);
              te();
              prof->n_gje_update++;
            } else {
              tb(&prof->gje_rhs_ms);
              launch_gje_premul(dg, ng, lv.maxn, ls);
              launch_gje_rhs(dg, lv.nsmall, lv.rhs_small, kRhsMaxN16, 0, nsteps, 0, ls, narrow);
              launch_gje_rhs(dg + lv.nsmall, ng - lv.nsmall, lv.rhs_large, lv.maxn, 0, nsteps, 0, ls, narrow);
              te();
              prof->n_gje_rhs++;
            }
          } else if (prof || (opt.noalloc && !gje_step_fits(lv.maxn))) {
            // panel and update on one stream (each launch timed when profiling)
            for (int k = 0; k < lv.maxn; k += kGjeNb) {
              tb(prof ? &prof->gje_panel_ms : nullptr);
              launch_gje_panel(dg, ng, k, lv.maxn, ls);
              te();
              tb(prof ? &prof->gje_update_ms : nullptr);
              launch_gje_update(dg, ng, k, lv.maxn, kGjeNb, 1 << 30, ls, rcol, lv.maxrhs);
              te();
              if (prof) {
                prof->n_gje_panel++;
                prof->n_gje_update++;
              }
            }
            if (!lv.rhs_in_step) {
              tb(prof ? &prof->gje_rhs_ms : nullptr);
              launch_gje_premul(dg, ng, lv.maxn, ls);
              launch_gje_rhs(dg, lv.nsmall, lv.rhs_small, kRhsMaxN16, 0, nsteps, 0, ls, narrow);
              launch_gje_rhs(dg + lv.nsmall, ng - lv.nsmall, lv.rhs_large, lv.maxn, 0, nsteps, 0, ls, narrow);
              te();
              if (prof) prof->n_gje_rhs++;
            }
          } else if (gje_step_fits(lv.maxn)) {
            // one launch per step: panel s with the update of step s - 1
            for (int st_i = 0; st_i < nsteps; ++st_i)
              launch_gje_step(dg, ng, st_i * kGjeNb, lv.maxn, ls, rcol, lv.maxrhs);
            if (lv.rhs_in_step) {  // the last step on the right-hand sides
              launch_gje_update(dg, ng, (nsteps - 1) * kGjeNb, lv.maxn, kGjeNb, 1 << 30, ls, rcol, lv.maxrhs);
            } else {
              launch_gje_premul(dg, ng, lv.maxn, ls);
              launch_gje_rhs(dg, lv.nsmall, lv.rhs_small, kRhsMaxN16, 0, nsteps, 0, ls, narrow);
              launch_gje_rhs(dg + lv.nsmall, ng - lv.nsmall, lv.rhs_large, lv.maxn, 0, nsteps, 0, ls, narrow);
            }
          } else {
            hipEvent_t rest1 = nullptr, rest2 = nullptr;  // updates of steps s - 1, s - 2
            for (int st_i = 0; st_i < nsteps; ++st_i) {
              const int k = st_i * kGjeNb;
              if (rest2) HIP_TRY(hipStreamWaitEvent(ls, rest2, 0));
              launch_gje_panel(dg, ng, k, lv.maxn, ls);
              hipEvent_t ep = ev_next();
              HIP_TRY(hipEventRecord(ep, ls));
              HIP_TRY(hipStreamWaitEvent(RN.aux_stream, ep, 0));
              launch_gje_update(dg, ng, k, lv.maxn, kGjeNb, 1 << 30, RN.aux_stream);
              hipEvent_t er = ev_next();
              HIP_TRY(hipEventRecord(er, RN.aux_stream));
              rest2 = rest1;
              rest1 = er;
            }
            if (rest1) HIP_TRY(hipStreamWaitEvent(ls, rest1, 0));
            launch_gje_premul(dg, ng, lv.maxn, ls);
            launch_gje_rhs(dg, lv.nsmall, lv.rhs_small, kRhsMaxN16, 0, nsteps, 0, ls, narrow);
            launch_gje_rhs(dg + lv.nsmall, ng - lv.nsmall, lv.rhs_large, lv.maxn, 0, nsteps, 0, ls, narrow);
          }
          if (prof) {
            double lu = 0.0, rhs = 0.0;
            for (const GjeDesc& G : lv.gje) {
              lu += 8.0 / 3.0 * (double)G.n * G.n * G.n;
              rhs += 8.0 * (double)G.n * G.n * (G.ncol - G.n);
            }
            if (gje_step_fits(lv.maxn))
              prof->gje_step_flops += lu + (lv.rhs_in_step ? rhs : 0.0);
            else
              prof->gje_panel_update_flops += lu;
            if (!lv.rhs_in_step) prof->gje_rhs_flops += rhs;
          }
          if (!lv.upd.empty()) {
            tb(prof ? &prof->sweep_gemm_ms : nullptr);
            launch_gemm(reinterpret_cast<GemmDesc*>(dbase + o_upd[l]), (int)lv.upd.size(), lv.upd_tiles, ls,
                        tune.gemm_slab_k);
            te();
            if (prof) {
              prof->n_sweep_gemm++;
              prof->sweep_gemm_flops += gemm_flops(lv.upd);
            }
          }
        }
        tb(prof ? &prof->backsub_ms : nullptr);
        for (int l = NL - 1; l >= 0; --l)
          launch_gemv_step(reinterpret_cast<GemvDesc*>(dbase + o_back[l]), (int)levels[l].back.size(), levels[l].backn,
                           rchunk, ls);
        te();
        if (prof) prof->n_backsub += NL;
        tb(prof ? &prof->bragg_ms : nullptr);
        if (!opt.adjoint) launch_bragg(d_ang, nang, ls);
        te();
        if (n_edst > 0)
          launch_gather_eta(reinterpret_cast<EtaSeg*>(dbase + o_eseg), max_seg, max_segn, reinterpret_cast<EtaDst*>(dbase + o_edst),
                            n_edst, ls);
      }
      HIP_TRY(hipGetLastError());

      return MLH_OK;
    };
    EvTimer T{st};
    static const bool no_graph = std::getenv("MLH_NO_GRAPH") != nullptr;
    if (prof || stop_phase != 0 || no_graph || opt.noalloc || opt.adjoint) {
      MLH_TRY(launch_all(st, T));
    } else {
      // every launch shape of the sequence: a cached graph is replayed only
      // when all of them, the workspace and its layout (which places the
      // descriptors and every system), are unchanged
      std::vector<int64_t> sig = {nb, nang, rchunk, (int64_t)doff, (int64_t)(intptr_t)wbase, asm_ls.tiles,
                                  asm_blk.tiles, gtiles, maxc, maxcols, maxncol, (int64_t)hq.size(),
                                  (int64_t)gs.size(), hq_small.n, hq_small.maxc, hq_small.maxncol, hq_large.maxc,
                                  hq_large.maxncol, tune.rhs_in_step_pct, tune.ls_row_blocks, tune.gje_rhs_cols,
                                  tune.asm_in_panels, tune.gemm_slab_k, n_edst, max_seg, max_segn, (int64_t)o_eseg, (int64_t)o_edst,
                                  (int64_t)(intptr_t)opt.tstamp, bi == 0 ? 1 : 0};
      for (int b = 0; b <= nb; ++b) sig.push_back((int64_t)sys_off[b]);
      for (const Level& lv : levels) {
        sig.push_back(lv.maxn);
        sig.push_back(lv.maxcol);
        sig.push_back(lv.maxrhs);
        sig.push_back(lv.nsmall);
        sig.push_back(lv.rhs_small);
        sig.push_back(lv.rhs_large);
        sig.push_back((int64_t)lv.gje.size());
        sig.push_back(lv.upd_tiles);
        sig.push_back((int64_t)lv.upd.size());
        sig.push_back(lv.backn);
        sig.push_back((int64_t)lv.back.size());
        sig.push_back(lv.rhs_in_step ? 1 : 0);
      }
      if (!(RN.gexec && RN.g_sig == sig)) {
        if (RN.gexec) {
          const hipError_t de = hipGraphExecDestroy(RN.gexec);
          RN.gexec = nullptr;
          HIP_TRY(de);
        }
        if (!RN.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&RN.cap_stream, hipStreamNonBlocking));
        // the capture stream waits for the descriptor upload
        hipEvent_t up;
        HIP_TRY(hipEventCreateWithFlags(&up, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(up, st));
        HIP_TRY(hipStreamWaitEvent(RN.cap_stream, up, 0));
        HIP_TRY(hipStreamSynchronize(RN.cap_stream));
        HIP_TRY(hipEventDestroy(up));
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(RN.cap_stream, hipStreamCaptureModeThreadLocal));
        mlh_status ls_ = launch_all(RN.cap_stream, T);
        hipError_t ce = hipStreamEndCapture(RN.cap_stream, &g);
        if (ls_ != MLH_OK || ce != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);  // the error already being reported is the one that matters
          if (ls_ != MLH_OK) return ls_;
          return fail(MLH_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        }
        hipError_t ie = hipGraphInstantiate(&RN.gexec, g, nullptr, nullptr, 0);
        const hipError_t gd = hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(MLH_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        HIP_TRY(gd);
        RN.g_sig = sig;
      }
      HIP_TRY(hipGraphLaunch(RN.gexec, st));
    }
    if (prof) HIP_TRY(T.collect());
    if (stop_phase != 0) {
      if (inspect) {
        inspect->dbg_R = V[0].W[0];
        inspect->dbg_S = V[0].S;
        inspect->dbg_RHS = V[0].RHS;
        inspect->dbg_eta = V[0].eta;
      }
      HIP_TRY(hipStreamSynchronize(st));
      return MLH_OK;
    }
    // ---- results (stream-ordered; the workspace of the next batch is
    //      written only after these copies)
    const hipMemcpyKind kind = opt.on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int b = 0; b < nb; ++b) {
      const int nK = SY(b).s->nK;
      const int64_t nden = SH(b).den_off[SH(b).I];
      for (int q = 0; q < R_of(b); ++q) {
        const int a = SY(b).ang[q];
        const AngleOut& o = outs[a];
        const cplx* src = V[b].out + (size_t)2 * nK * q;
        HIP_TRY(hipMemcpyAsync(o.aU, src, cbytes(nK), kind, st));
        HIP_TRY(hipMemcpyAsync(o.aD, src + nK, cbytes(nK), kind, st));
        if (o.orders)
          HIP_TRY(hipMemcpyAsync(o.orders, V[b].orders + (size_t)nK * q, sizeof(int) * nK, kind, st));
        if (opt.on_device && o.flux) HIP_TRY(hipMemcpyAsync(o.flux, V[b].flux + q, sizeof(double), kind, st));
        if (flux_to_host)
          HIP_TRY(hipMemcpyAsync(&h_flux[a], V[b].flux + q, sizeof(double), hipMemcpyDeviceToHost, st));
        if (eta_stage && o.eta)
          HIP_TRY(hipMemcpyAsync(o.eta, V[b].eta_rows + (size_t)nden * q, cbytes(nden), hipMemcpyDeviceToHost, st));
      }
    }
    if (opt.views) {
      SysViews& W = *opt.views;
      for (int b = 0; b < nb; ++b) {
        W.X.push_back(V[b].RHS);
        W.S.push_back(V[b].S);
        W.Th.push_back(V[b].Th);
        W.eta.push_back(V[b].eta);
        std::vector<int> ld;
        for (int j = 0; j <= SH(b).I; ++j) {
          int m, c, nc;
          layer_dims(SY(b).s, j, m, c, nc);
          ld.push_back(m + c);
        }
        W.ldX.push_back(ld);
      }
    }
    if (opt.keep_views && inspect && bi == 0) {
      inspect->dbg_R = V[0].W[0];
      inspect->dbg_S = V[0].S;
      inspect->dbg_RHS = V[0].RHS;
      inspect->dbg_eta = V[0].eta;
    }
    if (!opt.on_device) {
      int info[4] = {0, 0, 0, 0};
      HIP_TRY(hipMemcpyAsync(info, d_info, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (info[0] != 0) return fail(MLH_E_SINGULAR, "exact zero pivot in the block-tridiagonal solve");
    }
  }
  if (opt.on_device && flux_to_host) HIP_TRY(hipStreamSynchronize(st));
  return MLH_OK;
}

static bool theta_ok(double t) { return t > -kPi && t < 0.0; }

// mlh_solve and its variants on one stack: angles grouped by alpha, results
// at angle a of the caller's arrays
static mlh_status solve_impl(mlh_stack s, int32_t n_angles, const double* theta, double* aU, double* aD,
                             int32_t* orders, double* flux_err, double* eta, bool check_flux, const SolveOpts& opt) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  if (n_angles < 1 || !theta || !aU || !aD) return fail(MLH_E_INVALID_ARG, "mlh_solve: bad arguments");
  for (int a = 0; a < n_angles; ++a)
    if (!theta_ok(theta[a])) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  std::vector<SysSpec> sys;
  group_by_alpha(s, n_angles, theta, 0, sys);
  int64_t nden = 0;
  for (int v : s->n) nden += v;
  std::vector<AngleOut> outs(n_angles);
  for (int a = 0; a < n_angles; ++a) {
    AngleOut& o = outs[a];
    o.aU = aU + (size_t)2 * s->nK * a;
    o.aD = aD + (size_t)2 * s->nK * a;
    o.orders = orders ? orders + (size_t)s->nK * a : nullptr;
    o.flux = flux_err ? flux_err + a : nullptr;
    o.eta = eta ? eta + (size_t)2 * nden * a : nullptr;
  }
  const bool check = check_flux && s->flux_tol > 0;
  std::vector<double> h_flux;
  MLH_TRY(solve_systems(s->run, s->ctx, s->tune, sys, theta, outs, opt, !opt.on_device || check, h_flux, s));
  if (opt.stop_phase != 0) return MLH_OK;
  if (flux_err && !opt.on_device)
    for (int a = 0; a < n_angles; ++a) flux_err[a] = h_flux[a];
  if (check) {
    int worst = -1;
    for (int a = 0; a < n_angles; ++a)
      if (!(std::fabs(h_flux[a]) <= s->flux_tol) && (worst < 0 || !(std::fabs(h_flux[a]) <= std::fabs(h_flux[worst]))))
        worst = a;
    if (worst >= 0) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "flux error %.3e at angle %d exceeds the tolerance %.3e", h_flux[worst], worst,
                    s->flux_tol);
      return fail(MLH_E_ACCURACY, msg);
    }
  }
  return MLH_OK;
}

extern "C" mlh_status mlh_solve(mlh_stack s, int32_t n_angles, const double* theta, int32_t outputs_on_device,
                                double* aU, double* aD, int32_t* orders, double* flux_err, double* eta) {
  if (outputs_on_device != 0 && outputs_on_device != 1)
    return fail(MLH_E_INVALID_ARG, "mlh_solve: outputs_on_device must be 0 or 1");
  SolveOpts o;
  o.on_device = outputs_on_device == 1;
  return solve_impl(s, n_angles, theta, aU, aD, orders, flux_err, eta, true, o);
}

extern "C" mlh_status mlh_solve_noalloc(mlh_stack s, int32_t n_angles, const double* theta,
                                        int32_t outputs_on_device, double* aU, double* aD, int32_t* orders,
                                        double* flux_err, double* eta) {
  if (outputs_on_device != 0 && outputs_on_device != 1)
    return fail(MLH_E_INVALID_ARG, "mlh_solve_noalloc: outputs_on_device must be 0 or 1");
  SolveOpts o;
  o.on_device = outputs_on_device == 1;
  o.noalloc = true;
  return solve_impl(s, n_angles, theta, aU, aD, orders, flux_err, eta, true, o);
}

// ---------------------------------------------------------------------------
// field evaluation
// ---------------------------------------------------------------------------
extern "C" mlh_status mlh_field(mlh_stack s, double theta, int64_t n_pts, const double* x, const double* y,
                                int32_t outputs_on_device, double* u, int32_t* layer) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  if (!theta_ok(theta)) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  if (outputs_on_device != 0 && outputs_on_device != 1)
    return fail(MLH_E_INVALID_ARG, "mlh_field: outputs_on_device must be 0 or 1");
  if (n_pts < 0 || (n_pts > 0 && (!x || !y || !u))) return fail(MLH_E_INVALID_ARG, "mlh_field: bad arguments");
  for (int64_t t = 0; t < n_pts; ++t)
    if (!std::isfinite(x[t]) || !std::isfinite(y[t])) return fail(MLH_E_INVALID_ARG, "mlh_field: non-finite target");
  const int I = s->I, P = s->P, nK = s->nK;
  const double d = s->d;
  // ---- the solve, its workspace left in place
  std::vector<double> aU(2 * nK), aD(2 * nK), fl(1);
  std::vector<int32_t> ord(nK);
  {
    SolveOpts o;
    o.keep_views = true;
    MLH_TRY(solve_impl(s, 1, &theta, aU.data(), aD.data(), ord.data(), fl.data(), nullptr, false, o));
  }
  if (n_pts == 0) return MLH_OK;
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  // ---- targets into the unit cell, by region (-1 above U, layers, I+1 below D)
  const double ph = d * s->k[0] * std::cos(theta);  // alpha = e^{i ph}
  // (the interface heights cost a Fourier sum each, several per target:
  // chunks of targets on the host threads)
  std::vector<int> reg(n_pts);
  std::vector<FieldTarget> tg(n_pts);
  std::vector<int64_t> count(I + 3, 0);
  const int64_t chunk = 16384;
  parallel_for((int)((n_pts + chunk - 1) / chunk), [&](int c) {
    const int64_t t1 = std::min(n_pts, (int64_t)(c + 1) * chunk);
    for (int64_t t = (int64_t)c * chunk; t < t1; ++t) {
      const double m = std::floor((x[t] + 0.5 * d) / d);
      const double xc = x[t] - m * d;
      int r;
      if (y[t] >= s->yU) {
        r = -1;
      } else if (y[t] <= s->yD) {
        r = I + 1;
      } else {  // heights decrease with the interface index at every x
        int lo = 0, hi = I;  // first interface below the point
        while (lo < hi) {
          const int mid = (lo + hi) / 2;
          if (y[t] > s->curves[mid].height(xc))
            hi = mid;
          else
            lo = mid + 1;
        }
        r = lo;
      }
      reg[t] = r;
      FieldTarget& T = tg[t];
      T.x = xc;
      T.y = y[t];
      T.ph_re = std::cos(m * ph);
      T.ph_im = std::sin(m * ph);
      T.idx = t;
    }
  });
  for (int64_t t = 0; t < n_pts; ++t) ++count[reg[t] + 1];
  std::vector<int64_t> start(I + 4, 0);
  for (int r = 0; r < I + 3; ++r) start[r + 1] = start[r] + count[r];
  // order: by region, and inside a region by the cells of a grid of spacing
  // d/64 (row by row), so that the targets of a wavefront lie close together
  // and take the same branch of the Hankel routine for each source (two
  // stable counting sorts: by cell, then by region).  In the input order a
  // wavefront's lanes diverge over the series, recurrence and asymptotic
  // branches: a million random targets took 4.6 times as long.
  std::vector<int64_t> by_cell(n_pts);
  {
    const int gxn = 64;
    const double hx = d / gxn;
    double ylo = y[0], yhi = y[0];
    for (int64_t t = 1; t < n_pts; ++t) {
      ylo = std::min(ylo, y[t]);
      yhi = std::max(yhi, y[t]);
    }
    const int64_t rows = std::min<int64_t>(65536, std::max<int64_t>(1, n_pts / 64));  // grid rows at most
    const double hy = std::max(hx, (yhi - ylo) / (double)rows);
    const int64_t gyn = std::min<int64_t>((int64_t)((yhi - ylo) / hy) + 1, rows);
    std::vector<int64_t> cpos(gyn * gxn + 1, 0);
    std::vector<int32_t> cell(n_pts);
    for (int64_t t = 0; t < n_pts; ++t) {
      const int64_t cy = std::min<int64_t>(gyn - 1, (int64_t)((y[t] - ylo) / hy));
      const int cx = std::min(gxn - 1, std::max(0, (int)((tg[t].x + 0.5 * d) / hx)));
      cell[t] = (int32_t)(cy * gxn + cx);
      ++cpos[cell[t] + 1];
    }
    for (size_t c = 1; c < cpos.size(); ++c) cpos[c] += cpos[c - 1];
    for (int64_t t = 0; t < n_pts; ++t) by_cell[cpos[cell[t]]++] = t;
  }
  std::vector<FieldTarget> sorted(n_pts);
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t t : by_cell) sorted[pos[reg[t] + 1]++] = tg[t];
  }
  std::vector<FieldTile> tiles;
  for (int r = 0; r < I + 3; ++r)
    for (int64_t f = start[r]; f < start[r + 1]; f += 256)
      tiles.push_back(FieldTile{r, (int)f, (int)std::min<int64_t>(256, start[r + 1] - f)});
  if (n_pts > (int64_t)INT32_MAX - 256) return fail(MLH_E_UNSUPPORTED, "mlh_field: too many targets");
  // ---- device buffer: targets, tiles, regions, proxy jobs, strengths,
  //      amplitudes, and the outputs when the caller's are on the host
  Arena ar;
  const size_t o_tg = ar.reserve(sizeof(FieldTarget) * n_pts), o_ti = ar.reserve(sizeof(FieldTile) * tiles.size()),
               o_rg = ar.reserve(sizeof(FieldRegion) * (I + 3)), o_pj = ar.reserve(sizeof(ProxyStrengthJob) * (I + 1)),
               o_cf = ar.reserve(cbytes((size_t)(I + 1) * P)), o_am = ar.reserve(cbytes(2 * (size_t)nK)),
               o_u = outputs_on_device ? 0 : ar.reserve(cbytes(n_pts)),
               o_l = (outputs_on_device || !layer) ? 0 : ar.reserve(sizeof(int) * n_pts);
  char* buf = nullptr;
  hipError_t e = hipMalloc((void**)&buf, ar.off);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE, "mlh_field: allocation");
  struct Free {
    char* p;
    ~Free() { (void)hipFree(p); }
  } guard{buf};
  cplx* coef = reinterpret_cast<cplx*>(buf + o_cf);
  cplx* amp = reinterpret_cast<cplx*>(buf + o_am);
  std::vector<ProxyStrengthJob> pj(I + 1);
  std::vector<FieldRegion> rg(I + 3);
  for (int j = 0; j <= I; ++j) {
    int m, c, nc;
    layer_dims(s, j, m, c, nc);
    ProxyStrengthJob& J = pj[j];
    J.X = s->dbg_RHS[j];
    J.ldX = m + c;
    J.eta0 = j > 0 ? s->dbg_eta[j - 1] : s->dbg_eta[0];
    J.n0 = j > 0 ? s->n[j - 1] : s->n[0];
    J.eta1 = (j > 0 && j < I) ? s->dbg_eta[j] : nullptr;
    J.n1 = (j > 0 && j < I) ? s->n[j] : 0;
    J.c = coef + (size_t)j * P;
    J.P = P;
    FieldRegion& R = rg[j + 1];
    R.kind = 0;
    R.label = j;
    R.k = s->k[j];
    auto curve = [&](int i) {
      FieldCurve C{};
      if (i < 0 || i >= I) return C;
      C.x = s->gx[i];
      C.y = s->gy[i];
      C.nx = s->gnx[i];
      C.ny = s->gny[i];
      C.w = s->gw[i];
      C.eta = s->dbg_eta[i];
      C.y0 = s->curves[i].y0;
      C.N = s->N[i];
      return C;
    };
    R.above = curve(j - 1);
    R.below = curve(j);
    R.px = s->px[j];
    R.py = s->py[j];
    R.pnx = s->pnx[j];
    R.pny = s->pny[j];
    R.centre = s->centre[j];
    R.coef = J.c;
  }
  rg[0].kind = 1;
  rg[0].label = -1;
  rg[0].k = s->k[0];
  rg[0].amp = amp;
  rg[0].yline = s->yU;
  rg[I + 2].kind = 2;
  rg[I + 2].label = I + 1;
  rg[I + 2].k = s->k[I];
  rg[I + 2].amp = amp + nK;
  rg[I + 2].yline = s->yD;
  std::vector<double> amps(aU);
  amps.insert(amps.end(), aD.begin(), aD.end());
  HIP_TRY(hipMemcpyAsync(buf + o_tg, sorted.data(), sizeof(FieldTarget) * n_pts, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(buf + o_ti, tiles.data(), sizeof(FieldTile) * tiles.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(buf + o_rg, rg.data(), sizeof(FieldRegion) * rg.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(buf + o_pj, pj.data(), sizeof(ProxyStrengthJob) * pj.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(amp, amps.data(), cbytes(2 * (size_t)nK), hipMemcpyHostToDevice, st));
  FieldConsts fc{};
  fc.alpha_pow[0] = cpow_alpha(ph, -1);
  fc.alpha_pow[1] = cx(1.0, 0.0);
  fc.alpha_pow[2] = cpow_alpha(ph, 1);
  fc.d = d;
  fc.kappa0 = s->k[0] * std::cos(theta);
  fc.K = s->K;
  fc.nK = nK;
  fc.n0 = ord[0] + s->K;  // the solve's own order window
  fc.P = P;
  launch_proxy_strength(reinterpret_cast<ProxyStrengthJob*>(buf + o_pj), I + 1, st);
  double* ud = outputs_on_device ? u : reinterpret_cast<double*>(buf + o_u);
  int* ld = outputs_on_device ? layer : (layer ? reinterpret_cast<int*>(buf + o_l) : nullptr);
  launch_field(reinterpret_cast<FieldTile*>(buf + o_ti), (int)tiles.size(), reinterpret_cast<FieldRegion*>(buf + o_rg),
               reinterpret_cast<FieldTarget*>(buf + o_tg), ud, ld, fc, st);
  HIP_TRY(hipGetLastError());
  if (!outputs_on_device) {
    HIP_TRY(hipMemcpyAsync(u, ud, cbytes(n_pts), hipMemcpyDeviceToHost, st));
    if (layer) HIP_TRY(hipMemcpyAsync(layer, ld, sizeof(int) * n_pts, hipMemcpyDeviceToHost, st));
  }
  // the buffer is freed on return: wait for the work that reads it
  HIP_TRY(hipStreamSynchronize(st));
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// adjoint: gradient of the summed zeroth-order reflected efficiency
// ---------------------------------------------------------------------------
// the shape part of the adjoint (below): derivative pieces of the blocks that
// touch one smooth interface, in one shape coefficient, by central
// differences of the fill kernels at perturbed node geometry
// slot of the adjoint's device scratch, at least `bytes` long (a larger
// one replaces the old, which hipFree waits for)
static mlh_status adj_scratch(mlh_stack s, int slot, size_t bytes, char** out) {
  auto& b = s->adj_buf[slot];
  if (bytes > b.second) {
    if (b.first) HIP_TRY(hipFree(b.first));
    b = {nullptr, 0};
    const hipError_t e = hipMalloc((void**)&b.first, bytes);
    if (e != hipSuccess) {
      b = {nullptr, 0};
      return fail(e == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE, "mlh_adjoint: allocation");
    }
    b.second = bytes;
  }
  *out = b.first;
  return MLH_OK;
}

static mlh_status adjoint_shape(mlh_stack s, int32_t n_angles, const double* theta, const std::vector<SysSpec>& sys,
                                const std::vector<int64_t>& doff, const cplx* d_eta, const cplx* d_z, const cplx* d_c,
                                const cplx* d_l, const std::vector<size_t>& loff, size_t msum,
                                const std::vector<double>& aU, const std::vector<int>& q0, double* grad_shape);

extern "C" mlh_status mlh_adjoint(mlh_stack s, int32_t n_angles, const double* theta, double* J_out,
                                  double* grad_k, double* grad_shape) {
  if (!s || n_angles < 1 || !theta || !grad_k) return fail(MLH_E_INVALID_ARG, "mlh_adjoint: bad arguments");
  for (int a = 0; a < n_angles; ++a)
    if (!theta_ok(theta[a])) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  const int I = s->I, P = s->P, nK = s->nK;
  int64_t nden = 0;
  std::vector<int64_t> doff(I + 1, 0);
  for (int i = 0; i < I; ++i) doff[i + 1] = doff[i] + s->n[i];
  nden = doff[I];
  std::vector<SysSpec> sys;
  group_by_alpha(s, n_angles, theta, 0, sys);
  // ---- forward solve: amplitudes, order labels and densities on the host
  std::vector<double> aU((size_t)2 * nK * n_angles), aD(aU.size()), flux(n_angles);
  std::vector<int32_t> ord((size_t)nK * n_angles);
  std::vector<double> eta((size_t)2 * nden * n_angles);
  std::vector<AngleOut> outs(n_angles);
  for (int a = 0; a < n_angles; ++a)
    outs[a] = AngleOut{aU.data() + (size_t)2 * nK * a, aD.data() + (size_t)2 * nK * a, ord.data() + (size_t)nK * a,
                       flux.data() + a, eta.data() + (size_t)2 * nden * a};
  std::vector<double> h_flux;
  MLH_TRY(solve_systems(s->run, s->ctx, s->tune, sys, theta, outs, SolveOpts(), true, h_flux, nullptr));
  std::vector<int> q0(n_angles, -1);
  for (int a = 0; a < n_angles; ++a)
    for (int q = 0; q < nK; ++q)
      if (ord[(size_t)nK * a + q] == 0) q0[a] = q;
  for (int a = 0; a < n_angles; ++a)
    if (q0[a] < 0) return fail(MLH_E_INVALID_ARG, "mlh_adjoint: order 0 lies outside the Rayleigh-Bloch window");
  // ---- device buffers: forward densities, adjoint densities z, proxy
  //      strengths, v and l_w per layer, derivative pieces and their jobs
  std::vector<int> mrows(I + 1), crows(I + 1);
  size_t csum = 0, msum = 0;
  for (int j = 0; j <= I; ++j) {
    int m, c, nc;
    layer_dims(s, j, m, c, nc);
    mrows[j] = m;
    crows[j] = c;
    csum += c;
    msum += m;
  }
  size_t kb_extra = 0;
  for (int i = 0; i < I; ++i) kb_extra += (size_t)3 * s->n[i] * s->n[i];
  const size_t nacc = (size_t)n_angles * (I + 1);
  Arena ar;
  const size_t o_eta = ar.reserve(cbytes((size_t)nden * n_angles)), o_z = ar.reserve(cbytes((size_t)nden * n_angles)),
               o_c = ar.reserve(cbytes((size_t)n_angles * (I + 1) * P)), o_v = ar.reserve(cbytes(n_angles * csum)),
               o_l = ar.reserve(cbytes(n_angles * msum)), o_dum = ar.reserve(cbytes((size_t)2 * nK * n_angles)),
               o_acc = ar.reserve(sizeof(double) * 2 * nacc), o_dk = ar.reserve(s->dbytes),
               o_kb = ar.reserve(cbytes(kb_extra)), o_fj = ar.reserve(sizeof(FillJob) * s->h_fill.size()),
               o_sj = ar.reserve(sizeof(SelfJob) * 2 * s->h_self.size()),
               o_aj = ar.reserve(sizeof(AlpertJob) * 2 * s->h_alp.size());
  char* buf = nullptr;
  MLH_TRY(adj_scratch(s, 0, ar.off, &buf));
  cplx* d_eta = reinterpret_cast<cplx*>(buf + o_eta);
  cplx* d_z = reinterpret_cast<cplx*>(buf + o_z);
  cplx* d_c = reinterpret_cast<cplx*>(buf + o_c);
  cplx* d_v = reinterpret_cast<cplx*>(buf + o_v);
  cplx* d_l = reinterpret_cast<cplx*>(buf + o_l);
  double* d_acc = reinterpret_cast<double*>(buf + o_acc);
  char* dk = buf + o_dk;
  cplx* kb = reinterpret_cast<cplx*>(buf + o_kb);
  HIP_TRY(hipMemcpyAsync(d_eta, eta.data(), cbytes((size_t)nden * n_angles), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(d_acc, 0, sizeof(double) * 2 * nacc, st));
  // ---- derivative pieces dP/dk of every alpha-independent piece, at the
  //      same offsets as the pieces in the stack's arena; the self blocks
  //      have two (in k above and in k below the interface)
  auto mapc = [&](const cplx* p) -> cplx* {
    return p ? reinterpret_cast<cplx*>(dk + (reinterpret_cast<const char*>(p) - s->dmem)) : nullptr;
  };
  std::vector<FillJob> fj = s->h_fill;
  for (FillJob& F : fj) {
    F.dk = 1;
    for (int l = 0; l < 3; ++l) {
      F.out[l] = mapc(F.out[l]);
      F.out_t[l] = mapc(F.out_t[l]);
    }
  }
  std::vector<SelfJob> sj;
  std::vector<AlpertJob> aj;
  std::vector<cplx*> self_kb(I);
  {
    size_t off = 0;
    int tiles = 0, blocks = 0;
    for (int pass = 1; pass <= 2; ++pass)
      for (int i = 0; i < I; ++i) {
        SelfJob S = s->h_self[i];
        AlpertJob A = s->h_alp[i];
        S.dk = A.dk = pass;
        const size_t pe = (size_t)s->n[i] * s->n[i];
        for (int l = 0; l < 3; ++l) {
          S.out[l] = pass == 1 ? mapc(S.out[l]) : kb + off + l * pe;
          A.out[l] = S.out[l];
        }
        if (pass == 2) {
          self_kb[i] = kb + off;
          off += 3 * pe;
        }
        S.tile_begin = tiles;
        tiles += S.tiles_m * (S.tiles_m + 1) / 2;
        A.block_begin = blocks;
        blocks += A.N;
        sj.push_back(S);
        aj.push_back(A);
      }
    HIP_TRY(hipMemcpyAsync(buf + o_fj, fj.data(), sizeof(FillJob) * fj.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(buf + o_sj, sj.data(), sizeof(SelfJob) * sj.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(buf + o_aj, aj.data(), sizeof(AlpertJob) * aj.size(), hipMemcpyHostToDevice, st));
    launch_self(reinterpret_cast<SelfJob*>(buf + o_sj), (int)sj.size(), tiles, kAlpertA, st, true);
    launch_alpert(reinterpret_cast<AlpertJob*>(buf + o_aj), (int)aj.size(), blocks, kAlpertA, st, true);
    launch_fill(reinterpret_cast<FillJob*>(buf + o_fj), (int)fj.size(), s->fill_tiles, st, true);
    HIP_TRY(hipGetLastError());
  }
  // ---- adjoint solve: A'^T z = w; z lands in the density rows of d_z, the
  //      workspace keeps X, the least-squares factors and z
  SysViews views;
  {
    std::vector<AngleOut> o2(n_angles);
    cplx* dum = reinterpret_cast<cplx*>(buf + o_dum);
    for (int a = 0; a < n_angles; ++a)
      o2[a] = AngleOut{reinterpret_cast<double*>(dum + (size_t)2 * nK * a),
                       reinterpret_cast<double*>(dum + (size_t)2 * nK * a + nK), nullptr, nullptr,
                       reinterpret_cast<double*>(d_z + (size_t)nden * a)};
    SolveOpts o;
    o.on_device = true;
    o.adjoint = true;
    o.adj_q0 = &q0;
    o.views = &views;
    std::vector<double> hf;
    MLH_TRY(solve_systems(s->run, s->ctx, s->tune, sys, theta, o2, o, false, hf, nullptr));
  }
  // ---- per angle: proxy strengths, v_j, l_w,j, and the contractions
  std::vector<ProxyStrengthJob> pj;
  std::vector<BtzJob> bj;
  std::vector<LsAdjJob> lj;
  std::vector<BilinJob> blj;
  int btiles = 0;
  std::vector<size_t> voff(I + 1), loff(I + 1);
  {
    size_t vo = 0, lo = 0;
    for (int j = 0; j <= I; ++j) {
      voff[j] = vo;
      loff[j] = lo;
      vo += crows[j];
      lo += mrows[j];
    }
  }
  auto bil = [&](const cplx* const* P, const cplx* coef, int np, int rows, int cols, int ld, const cplx* left,
                 const cplx* right, double scale, int out) {
    BilinJob B{};
    for (int p = 0; p < np; ++p) {
      B.P[p] = P[p];
      B.coef[p] = coef[p];
    }
    B.np = np;
    B.rows = rows;
    B.cols = cols;
    B.ld = ld;
    B.left = left;
    B.right = right;
    B.scale = scale;
    B.out = out;
    B.tile_begin = btiles;
    btiles += ((rows + 63) / 64) * ((cols + 63) / 64);
    blj.push_back(B);
  };
  const cplx one = cx(1.0, 0.0);
  for (size_t b = 0; b < sys.size(); ++b)
    for (size_t q = 0; q < sys[b].ang.size(); ++q) {
      const int a = sys[b].ang[q];
      const cplx* eta_a = d_eta + (size_t)nden * a;
      (void)eta_a;
      const cplx* z_a = d_z + (size_t)nden * a;
      cplx* c_a = d_c + (size_t)a * (I + 1) * P;
      cplx* v_a = d_v + (size_t)a * csum;
      cplx* l_a = d_l + (size_t)a * msum;
      for (int j = 0; j <= I; ++j) {
        ProxyStrengthJob J{};
        J.X = views.X[b][j];
        J.ldX = views.ldX[b][j];
        J.eta0 = j > 0 ? eta_a + doff[j - 1] : eta_a;
        J.n0 = j > 0 ? s->n[j - 1] : s->n[0];
        J.eta1 = (j > 0 && j < I) ? eta_a + doff[j] : nullptr;
        J.n1 = (j > 0 && j < I) ? s->n[j] : 0;
        J.c = c_a + (size_t)j * P;
        J.P = P;
        pj.push_back(J);
        BtzJob Bz{};
        if (j < I) {
          Bz.B1 = s->B_own[j];
          Bz.ld1 = s->n[j];
          Bz.z1 = z_a + doff[j];
          Bz.n1 = s->n[j];
        }
        if (j > 0) {
          Bz.B2 = s->B_below[j - 1];
          Bz.ld2 = s->n[j - 1];
          Bz.z2 = z_a + doff[j - 1];
          Bz.n2 = s->n[j - 1];
        }
        Bz.v = v_a + voff[j];
        Bz.P = P;
        Bz.c = crows[j];
        Bz.unit = j == 0 ? P + q0[a] : -1;
        bj.push_back(Bz);
        LsAdjJob L{};
        L.S = views.S[b][j];
        L.T = views.Th[b][j];
        L.v = v_a + voff[j];
        L.ell = l_a + loff[j];
        L.M = mrows[j] + crows[j];
        L.m = mrows[j];
        L.c = crows[j];
        lj.push_back(L);
      }
      // contractions, accumulated at acc[a (I+1) + layer]: density rows with
      // left = z (= -l_eta), wall rows with left = l_w and scale -1
      const double ph = s->d * s->k[0] * std::cos(theta[a]);
      const cplx am1 = cpow_alpha(ph, -1), ap1 = cpow_alpha(ph, 1), am2 = cpow_alpha(ph, -2);
      const cplx c3[3] = {am1, one, ap1};
      const cplx cC[2] = {am2, cx(-ap1.re, -ap1.im)};
      const cplx cQ[2] = {am1, cx(-1.0, 0.0)};
      const int base = a * (I + 1);
      for (int i = 0; i < I; ++i) {
        const int n = s->n[i];
        const size_t pe = (size_t)n * n;
        const cplx* zi = z_a + doff[i];
        const cplx* ei = eta_a + doff[i];
        const cplx* sa[3] = {mapc(s->A_self[i]), mapc(s->A_self[i]) + pe, mapc(s->A_self[i]) + 2 * pe};
        bil(sa, c3, 3, n, n, n, zi, ei, 1.0, base + i);
        const cplx* sb[3] = {self_kb[i], self_kb[i] + pe, self_kb[i] + 2 * pe};
        bil(sb, c3, 3, n, n, n, zi, ei, 1.0, base + i + 1);
        if (i + 1 < I) {
          const int n1 = s->n[i + 1];
          const size_t pu = (size_t)n * n1;
          const cplx* su[3] = {mapc(s->A_up[i]), mapc(s->A_up[i]) + pu, mapc(s->A_up[i]) + 2 * pu};
          bil(su, c3, 3, n, n1, n, zi, eta_a + doff[i + 1], 1.0, base + i + 1);
          const cplx* sd[3] = {mapc(s->A_dn[i]), mapc(s->A_dn[i]) + pu, mapc(s->A_dn[i]) + 2 * pu};
          bil(sd, c3, 3, n1, n, n1, z_a + doff[i + 1], ei, 1.0, base + i + 1);
        }
        const cplx* bo[1] = {mapc(s->B_own[i])};
        bil(bo, &one, 1, n, P, n, zi, c_a + (size_t)i * P, 1.0, base + i);
        const cplx* bb[1] = {mapc(s->B_below[i])};
        bil(bb, &one, 1, n, P, n, zi, c_a + (size_t)(i + 1) * P, 1.0, base + i + 1);
      }
      const int mw2 = 2 * s->Mw, mud2 = 2 * s->Mud;
      for (int j = 0; j <= I; ++j) {
        const cplx* lw = l_a + loff[j];
        if (j > 0) {
          const size_t ea = (size_t)mw2 * s->n[j - 1];
          const cplx* ca[2] = {mapc(s->C_above[j]), mapc(s->C_above[j]) + ea};
          bil(ca, cC, 2, mw2, s->n[j - 1], mw2, lw, eta_a + doff[j - 1], -1.0, base + j);
        }
        if (j < I) {
          const size_t eo = (size_t)mw2 * s->n[j];
          const cplx* co[2] = {mapc(s->C_own[j]), mapc(s->C_own[j]) + eo};
          bil(co, cC, 2, mw2, s->n[j], mw2, lw, eta_a + doff[j], -1.0, base + j);
        }
        const size_t qe = (size_t)mw2 * P;
        const cplx* sq[2] = {mapc(s->Q[j]), mapc(s->Q[j]) + qe};
        bil(sq, cQ, 2, mw2, P, mw2, lw, c_a + (size_t)j * P, -1.0, base + j);
      }
      {  // the rows on D (radiation condition of the bottom layer)
        const cplx* lw = l_a + loff[I] + mw2;
        const size_t ze = (size_t)mud2 * s->n[I - 1];
        const cplx* zd[3] = {mapc(s->Z_D), mapc(s->Z_D) + ze, mapc(s->Z_D) + 2 * ze};
        bil(zd, c3, 3, mud2, s->n[I - 1], mud2, lw, eta_a + doff[I - 1], -1.0, base + I);
        const cplx* vd[1] = {mapc(s->V_D)};
        bil(vd, &one, 1, mud2, P, mud2, lw, c_a + (size_t)I * P, -1.0, base + I);
      }
    }
  Arena ja;
  const size_t o_pj = ja.reserve(sizeof(ProxyStrengthJob) * pj.size()), o_bj = ja.reserve(sizeof(BtzJob) * bj.size()),
               o_lj = ja.reserve(sizeof(LsAdjJob) * lj.size()), o_blj = ja.reserve(sizeof(BilinJob) * blj.size());
  char* jbuf = nullptr;
  MLH_TRY(adj_scratch(s, 1, ja.off, &jbuf));
  HIP_TRY(hipMemcpyAsync(jbuf + o_pj, pj.data(), sizeof(ProxyStrengthJob) * pj.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(jbuf + o_bj, bj.data(), sizeof(BtzJob) * bj.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(jbuf + o_lj, lj.data(), sizeof(LsAdjJob) * lj.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(jbuf + o_blj, blj.data(), sizeof(BilinJob) * blj.size(), hipMemcpyHostToDevice, st));
  launch_proxy_strength(reinterpret_cast<ProxyStrengthJob*>(jbuf + o_pj), (int)pj.size(), st);
  launch_btz(reinterpret_cast<BtzJob*>(jbuf + o_bj), (int)bj.size(), st);
  launch_ls_adjoint(reinterpret_cast<LsAdjJob*>(jbuf + o_lj), (int)lj.size(), st);
  launch_bilinear(reinterpret_cast<BilinJob*>(jbuf + o_blj), (int)blj.size(), btiles, d_acc, st);
  HIP_TRY(hipGetLastError());
  std::vector<double> acc(2 * nacc);
  std::vector<double> lD((size_t)2 * n_angles * 2 * s->Mud);
  HIP_TRY(hipMemcpyAsync(acc.data(), d_acc, sizeof(double) * acc.size(), hipMemcpyDeviceToHost, st));
  for (int a = 0; a < n_angles; ++a)
    HIP_TRY(hipMemcpyAsync(lD.data() + (size_t)2 * a * 2 * s->Mud, d_l + (size_t)a * msum + loff[I] + 2 * s->Mw,
                           cbytes(2 * (size_t)s->Mud), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // ---- gradient: dJ/dk_j = sum_a 2 Re(conj(a0) da0/dk_j); the rows on D
  //      also hold W_D = -[e; -i k^D e] (eq. (59)), whose second half moves
  //      with k_{I+1}: d(i k^D_n)/dk = i k/k^D_n
  double Jsum = 0.0;
  for (int j = 0; j <= I; ++j) grad_k[j] = 0.0;
  grad_k[0] = std::nan("");
  for (int a = 0; a < n_angles; ++a) {
    const double a0r = aU[(size_t)2 * nK * a + 2 * q0[a]], a0i = aU[(size_t)2 * nK * a + 2 * q0[a] + 1];
    Jsum += a0r * a0r + a0i * a0i;
    auto add = [&](int j, double dr, double di) { grad_k[j] += 2.0 * (a0r * dr + a0i * di); };
    for (int j = 1; j <= I; ++j) add(j, acc[2 * ((size_t)a * (I + 1) + j)], acc[2 * ((size_t)a * (I + 1) + j) + 1]);
    const double kI = s->k[I];
    const double kap0 = s->k[0] * std::cos(theta[a]);
    double wr = 0.0, wi = 0.0;  // l_D2^T dW a^D
    for (int q = 0; q < nK; ++q) {
      const int nq = ord[(size_t)nK * a + q];
      const double kap = kap0 + 2.0 * kPi * nq / s->d;
      const double kk = kI * kI - kap * kap;
      if (std::fabs(kk) <= 1e-14 * kI * kI) continue;  // grazing order: no derivative
      // i k/k^D_n: k^D real (propagating) or i|.| (evanescent)
      double fr, fi;
      if (kk > 0) {
        fr = 0.0;
        fi = kI / std::sqrt(kk);
      } else {
        fr = kI / std::sqrt(-kk);
        fi = 0.0;
      }
      const double adr = aD[(size_t)2 * nK * a + 2 * q], adi = aD[(size_t)2 * nK * a + 2 * q + 1];
      const double gr = fr * adr - fi * adi, gi = fr * adi + fi * adr;  // f a^D_n
      for (int mm = 0; mm < s->Mud; ++mm) {
        const double x = -0.5 * s->d + s->d * (mm + 0.5) / s->Mud;
        const double er = std::cos(kap * x), ei = std::sin(kap * x);
        const double tr = er * gr - ei * gi, ti = er * gi + ei * gr;
        const double lr = lD[(size_t)2 * a * 2 * s->Mud + 2 * (s->Mud + mm)];
        const double li = lD[(size_t)2 * a * 2 * s->Mud + 2 * (s->Mud + mm) + 1];
        wr += lr * tr - li * ti;
        wi += lr * ti + li * tr;
      }
    }
    add(I, -wr, -wi);
  }
  if (J_out) *J_out = Jsum;
  if (grad_shape)
    MLH_TRY(adjoint_shape(s, n_angles, theta, sys, doff, d_eta, d_z, d_c, d_l, loff, msum, aU, q0, grad_shape));
  return MLH_OK;
}

static mlh_status adjoint_shape(mlh_stack s, int32_t n_angles, const double* theta, const std::vector<SysSpec>& sys,
                                const std::vector<int64_t>& doff, const cplx* d_eta, const cplx* d_z, const cplx* d_c,
                                const cplx* d_l, const std::vector<size_t>& loff, size_t msum,
                                const std::vector<double>& aU, const std::vector<int>& q0, double* grad_shape) {
  hipStream_t st = s->ctx->stream;
  const int I = s->I, P = s->P, nK = s->nK;
  const int64_t nden = doff[I];
  const int mw2 = 2 * s->Mw, mud2 = 2 * s->Mud;
  // the parameters: cos then sin coefficients of every smooth interface
  struct Par {
    int i, m, sinpart;
    int64_t out;
  };
  std::vector<Par> par;
  int64_t nout = 0;
  for (int i = 0; i < I; ++i) {
    const HostCurve& c = s->curves[i];
    if (c.cornered) continue;
    const int nm = (int)c.prof.om.size();
    for (int sp = 0; sp < 2; ++sp)
      for (int m = 0; m < nm; ++m) par.push_back(Par{i, m, sp, nout + sp * nm + m});
    nout += 2 * nm;
  }
  for (int64_t t = 0; t < nout; ++t) grad_shape[t] = 0.0;
  if (par.empty()) return MLH_OK;
  // central differences in the coefficient: step relative to the profile's size
  double hstep = 1e-6;
  {
    double amp = 0.0;
    for (int i = 0; i < I; ++i)
      for (double v : s->curves[i].prof.ca) amp = std::max(amp, std::fabs(v));
    for (int i = 0; i < I; ++i)
      for (double v : s->curves[i].prof.sa) amp = std::max(amp, std::fabs(v));
    if (amp > 0) hstep = 1e-5 * std::max(amp, 1e-3 * s->d);
  }
  // adjoint densities z of interface 1 on the host (right-hand-side term)
  std::vector<double> z1((size_t)2 * s->n[0] * n_angles);
  for (int a = 0; a < n_angles; ++a)
    HIP_TRY(hipMemcpyAsync(z1.data() + (size_t)2 * s->n[0] * a, d_z + (size_t)nden * a, cbytes(s->n[0]),
                           hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int chunk = 32;  // parameters per pass (two perturbed geometries each)
  // the perturbed curves of the pass starting at parameter q0, on host
  // threads (each curve with its Alpert auxiliary invariants costs
  // milliseconds); the next pass's curves are built while this pass runs
  auto build_pass = [&](size_t q0, std::vector<HostCurve>& out) {
    const int nq = (int)std::min(par.size() - q0, (size_t)chunk);
    out.assign(2 * nq, HostCurve());
    parallel_for(2 * nq, [&](int t) {
      const Par& pp = par[q0 + t / 2];
      const HostCurve& c0 = s->curves[pp.i];
      std::vector<double> ca(c0.prof.ca), sa(c0.prof.sa);
      (pp.sinpart ? sa : ca)[pp.m] += (t % 2 == 0 ? 1.0 : -1.0) * hstep;
      mlh_interface in{};
      in.kind = MLH_IFACE_FOURIER;
      in.y0 = c0.y0;
      in.n_modes = (int)ca.size();
      in.cos_coef = ca.data();
      in.sin_coef = sa.data();
      in.n_nodes = c0.N;
      build_fourier_curve(in, s->d, out[t]);  // writes out[t] only
    });
  };
  std::vector<HostCurve> cur, next;
  build_pass(0, cur);
  for (size_t p0 = 0; p0 < par.size(); p0 += chunk, cur.swap(next)) {
    const int np_ = (int)std::min(par.size() - p0, (size_t)chunk);
    struct Joiner {  // joined on every way out of the pass, early returns included
      std::thread th;
      ~Joiner() {
        if (th.joinable()) th.join();
      }
    } prefetch;
    if (p0 + chunk < par.size()) prefetch.th = std::thread([&, p0]() { build_pass(p0 + chunk, next); });
    // ---- perturbed geometry and the pieces of the blocks that touch it
    Arena ar;
    std::vector<size_t> o_geo(2 * np_), o_aux(2 * np_);
    for (int t = 0; t < 2 * np_; ++t) {
      const int N = s->curves[par[p0 + t / 2].i].N;
      o_geo[t] = ar.reserve(sizeof(double) * 5 * N);
      o_aux[t] = ar.reserve(sizeof(double) * 6 * (size_t)N * kAlpertAux);
    }
    const size_t o_geo_end = ar.off;
    // jobs: for every perturbation, the self and Alpert jobs of its interface
    // and the fill jobs whose targets or sources lie on it, with the
    // perturbed geometry and outputs in scratch pieces of the same shapes
    std::vector<std::map<const cplx*, size_t>> omap(2 * np_);
    auto scratch = [&](int t, const cplx* orig, size_t elems) -> size_t {
      auto it = omap[t].find(orig);
      if (it != omap[t].end()) return it->second;
      const size_t o = ar.reserve(cbytes(elems));
      omap[t][orig] = o;
      return o;
    };
    struct FJ {
      FillJob J;
      int t;
      size_t out[3], out_t[3];
    };
    std::vector<FJ> fjobs;
    std::vector<std::pair<SelfJob, int>> sjobs;
    std::vector<std::pair<AlpertJob, int>> ajobs;
    std::vector<size_t> sout(2 * np_);
    for (int t = 0; t < 2 * np_; ++t) {
      const int i = par[p0 + t / 2].i;
      const int n = s->n[i];
      sout[t] = scratch(t, s->A_self[i], (size_t)3 * n * n);
      for (const FillJob& F : s->h_fill) {
        const bool tg = F.tx == s->gx[i], sr = F.sx == s->gx[i];
        if (!tg && !sr) continue;
        FJ f{F, t, {0, 0, 0}, {0, 0, 0}};
        const size_t cols = F.kind == kFillProxy ? (size_t)F.Ns : (size_t)2 * F.Ns;
        for (int l = 0; l < F.npieces; ++l) f.out[l] = scratch(t, F.out[l], (size_t)F.ld * cols);
        if (F.kind == kFillPair)
          for (int l = 0; l < F.npieces; ++l) f.out_t[l] = scratch(t, F.out_t[l], (size_t)F.ld_t * 2 * F.Mt);
        fjobs.push_back(f);
      }
    }
    const size_t o_fj = ar.reserve(sizeof(FillJob) * fjobs.size()),
                 o_sj = ar.reserve(sizeof(SelfJob) * 2 * np_), o_aj = ar.reserve(sizeof(AlpertJob) * 2 * np_);
    char* buf = nullptr;
    MLH_TRY(adj_scratch(s, 2, ar.off, &buf));  // the previous pass ended with a stream wait
    auto dp = [&](size_t o) { return reinterpret_cast<double*>(buf + o); };
    auto cpp = [&](size_t o) { return reinterpret_cast<cplx*>(buf + o); };
    // the geometry of every perturbed curve, laid out as in the arena (it
    // opens the arena), goes over in one copy
    std::vector<double> hb(o_geo_end / sizeof(double));
    for (int t = 0; t < 2 * np_; ++t) {
      const HostCurve& c = cur[t];
      double* g = hb.data() + o_geo[t] / sizeof(double);
      for (auto* v : {&c.x, &c.y, &c.nx, &c.ny, &c.w}) g = std::copy(v->begin(), v->end(), g);
      double* x = hb.data() + o_aux[t] / sizeof(double);
      for (auto* v : {&c.ar2, &c.and_, &c.anpd, &c.ann, &c.acw, &c.at}) x = std::copy(v->begin(), v->end(), x);
    }
    HIP_TRY(hipMemcpyAsync(buf, hb.data(), o_geo_end, hipMemcpyHostToDevice, st));
    std::vector<FillJob> fj;
    std::vector<SelfJob> sj;
    std::vector<AlpertJob> aj;
    int ftiles = 0, stiles = 0, ablocks = 0;
    for (int t = 0; t < 2 * np_; ++t) {
      const int i = par[p0 + t / 2].i;
      const int N = s->N[i];
      const double* gx = dp(o_geo[t]);
      const double *gy = gx + N, *gnx = gx + 2 * N, *gny = gx + 3 * N, *gw = gx + 4 * N;
      const size_t na = (size_t)N * kAlpertAux;
      const double* ax = dp(o_aux[t]);
      SelfJob S = s->h_self[i];
      S.x = gx;
      S.y = gy;
      S.nx = gnx;
      S.ny = gny;
      S.w = gw;
      const size_t pe = (size_t)s->n[i] * s->n[i];
      for (int l = 0; l < 3; ++l) S.out[l] = cpp(sout[t]) + l * pe;
      S.tile_begin = stiles;
      stiles += S.tiles_m * (S.tiles_m + 1) / 2;
      sj.push_back(S);
      AlpertJob A = s->h_alp[i];
      A.r2 = ax;
      A.nd = ax + na;
      A.npd = ax + 2 * na;
      A.nn = ax + 3 * na;
      A.cw = ax + 4 * na;
      A.t = ax + 5 * na;
      for (int l = 0; l < 3; ++l) A.out[l] = S.out[l];
      A.block_begin = ablocks;
      ablocks += A.N;
      aj.push_back(A);
    }
    for (FJ& f : fjobs) {
      FillJob J = f.J;
      const int i = par[p0 + f.t / 2].i;
      const int N = s->N[i];
      const double* gx = dp(o_geo[f.t]);
      if (J.tx == s->gx[i]) {
        J.tx = gx;
        J.ty = gx + N;
        J.tnx = gx + 2 * N;
        J.tny = gx + 3 * N;
        if (J.kind == kFillPair) J.tw = gx + 4 * N;
      }
      if (J.sx == s->gx[i]) {
        J.sx = gx;
        J.sy = gx + N;
        J.snx = gx + 2 * N;
        J.sny = gx + 3 * N;
        J.sw = gx + 4 * N;
      }
      for (int l = 0; l < J.npieces; ++l) {
        J.out[l] = cpp(f.out[l]);
        if (J.kind == kFillPair) J.out_t[l] = cpp(f.out_t[l]);
      }
      J.dk = 0;
      const int tm = J.kind == kFillPair ? kSelfTile : kFillTileM, tn = J.kind == kFillPair ? kSelfTile : kFillTileN;
      J.tile_begin = ftiles;
      ftiles += J.tiles_m * ((J.Ns + tn - 1) / tn);
      (void)tm;
      fj.push_back(J);
    }
    HIP_TRY(hipMemcpyAsync(buf + o_fj, fj.data(), sizeof(FillJob) * fj.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(buf + o_sj, sj.data(), sizeof(SelfJob) * sj.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(buf + o_aj, aj.data(), sizeof(AlpertJob) * aj.size(), hipMemcpyHostToDevice, st));
    launch_self(reinterpret_cast<SelfJob*>(buf + o_sj), (int)sj.size(), stiles, kAlpertA, st);
    launch_alpert(reinterpret_cast<AlpertJob*>(buf + o_aj), (int)aj.size(), ablocks, kAlpertA, st);
    launch_fill(reinterpret_cast<FillJob*>(buf + o_fj), (int)fj.size(), ftiles, st);
    HIP_TRY(hipGetLastError());
    // ---- contractions: (P+ - P-)/2h of every touched block with the adjoint
    //      and forward vectors, per angle and parameter
    std::vector<BilinJob> blj;
    int btiles = 0;
    const size_t nacc = (size_t)n_angles * np_;
    auto bil = [&](int pidx, int a, const cplx* const* Pp, const cplx* const* Pm, const cplx* coef, int np, int rows,
                   int cols, int ld, const cplx* left, const cplx* right, double scale) {
      BilinJob B{};
      const double ih = 0.5 / hstep;
      for (int q = 0; q < np; ++q) {
        B.P[q] = Pp[q];
        B.coef[q] = cx(coef[q].re * ih, coef[q].im * ih);
        B.P[np + q] = Pm[q];
        B.coef[np + q] = cx(-coef[q].re * ih, -coef[q].im * ih);
      }
      B.np = 2 * np;
      B.rows = rows;
      B.cols = cols;
      B.ld = ld;
      B.left = left;
      B.right = right;
      B.scale = scale;
      B.out = (int)((size_t)a * np_ + pidx);
      B.tile_begin = btiles;
      btiles += ((rows + 63) / 64) * ((cols + 63) / 64);
      blj.push_back(B);
    };
    const cplx one = cx(1.0, 0.0);
    for (int pidx = 0; pidx < np_; ++pidx) {
      const int i = par[p0 + pidx].i;
      const int tp = 2 * pidx, tm_ = 2 * pidx + 1;
      auto piece = [&](int t, const cplx* orig) { return cpp(omap[t].at(orig)); };
      for (int a = 0; a < n_angles; ++a) {
        const cplx* eta_a = d_eta + (size_t)nden * a;
        const cplx* z_a = d_z + (size_t)nden * a;
        const cplx* c_a = d_c + (size_t)a * (I + 1) * P;
        const cplx* l_a = d_l + (size_t)a * msum;
        const double ph = s->d * s->k[0] * std::cos(theta[a]);
        const cplx am1 = cpow_alpha(ph, -1), ap1 = cpow_alpha(ph, 1), am2 = cpow_alpha(ph, -2);
        const cplx c3[3] = {am1, one, ap1};
        const cplx cC[2] = {am2, cx(-ap1.re, -ap1.im)};
        const int n = s->n[i];
        const size_t pe = (size_t)n * n;
        {
          const cplx* pp[3] = {cpp(sout[tp]), cpp(sout[tp]) + pe, cpp(sout[tp]) + 2 * pe};
          const cplx* pm[3] = {cpp(sout[tm_]), cpp(sout[tm_]) + pe, cpp(sout[tm_]) + 2 * pe};
          bil(pidx, a, pp, pm, c3, 3, n, n, n, z_a + doff[i], eta_a + doff[i], 1.0);
        }
        auto pair3 = [&](const cplx* base, size_t pel, int rows, int cols, const cplx* left, const cplx* right) {
          const cplx* pp[3] = {piece(tp, base), piece(tp, base + pel), piece(tp, base + 2 * pel)};
          const cplx* pm[3] = {piece(tm_, base), piece(tm_, base + pel), piece(tm_, base + 2 * pel)};
          bil(pidx, a, pp, pm, c3, 3, rows, cols, rows, left, right, 1.0);
        };
        if (i > 0) {
          const size_t pu = (size_t)s->n[i - 1] * n;
          pair3(s->A_up[i - 1], pu, s->n[i - 1], n, z_a + doff[i - 1], eta_a + doff[i]);
          pair3(s->A_dn[i - 1], pu, n, s->n[i - 1], z_a + doff[i], eta_a + doff[i - 1]);
        }
        if (i + 1 < I) {
          const size_t pu = (size_t)n * s->n[i + 1];
          pair3(s->A_up[i], pu, n, s->n[i + 1], z_a + doff[i], eta_a + doff[i + 1]);
          pair3(s->A_dn[i], pu, s->n[i + 1], n, z_a + doff[i + 1], eta_a + doff[i]);
        }
        {
          const cplx* pp[1] = {piece(tp, s->B_own[i])};
          const cplx* pm[1] = {piece(tm_, s->B_own[i])};
          bil(pidx, a, pp, pm, &one, 1, n, P, n, z_a + doff[i], c_a + (size_t)i * P, 1.0);
          const cplx* qp[1] = {piece(tp, s->B_below[i])};
          const cplx* qm[1] = {piece(tm_, s->B_below[i])};
          bil(pidx, a, qp, qm, &one, 1, n, P, n, z_a + doff[i], c_a + (size_t)(i + 1) * P, 1.0);
        }
        {  // walls of the layers above (i) and below (i + 1) the interface
          const size_t eo = (size_t)mw2 * n;
          const cplx* pp[2] = {piece(tp, s->C_own[i]), piece(tp, s->C_own[i] + eo)};
          const cplx* pm[2] = {piece(tm_, s->C_own[i]), piece(tm_, s->C_own[i] + eo)};
          bil(pidx, a, pp, pm, cC, 2, mw2, n, mw2, l_a + loff[i], eta_a + doff[i], -1.0);
          const cplx* qp[2] = {piece(tp, s->C_above[i + 1]), piece(tp, s->C_above[i + 1] + eo)};
          const cplx* qm[2] = {piece(tm_, s->C_above[i + 1]), piece(tm_, s->C_above[i + 1] + eo)};
          bil(pidx, a, qp, qm, cC, 2, mw2, n, mw2, l_a + loff[i + 1], eta_a + doff[i], -1.0);
        }
        const size_t ze = (size_t)mud2 * n;
        if (i == 0) {
          const cplx* pp[3] = {piece(tp, s->Z_U), piece(tp, s->Z_U + ze), piece(tp, s->Z_U + 2 * ze)};
          const cplx* pm[3] = {piece(tm_, s->Z_U), piece(tm_, s->Z_U + ze), piece(tm_, s->Z_U + 2 * ze)};
          bil(pidx, a, pp, pm, c3, 3, mud2, n, mud2, l_a + loff[0] + mw2, eta_a + doff[0], -1.0);
        }
        if (i == I - 1) {
          const cplx* pp[3] = {piece(tp, s->Z_D), piece(tp, s->Z_D + ze), piece(tp, s->Z_D + 2 * ze)};
          const cplx* pm[3] = {piece(tm_, s->Z_D), piece(tm_, s->Z_D + ze), piece(tm_, s->Z_D + 2 * ze)};
          bil(pidx, a, pp, pm, c3, 3, mud2, n, mud2, l_a + loff[I] + mw2, eta_a + doff[I - 1], -1.0);
        }
      }
    }
    Arena jb;
    const size_t o_b = jb.reserve(sizeof(BilinJob) * blj.size()), o_acc = jb.reserve(sizeof(double) * 2 * nacc);
    char* jbuf = nullptr;
    MLH_TRY(adj_scratch(s, 3, jb.off, &jbuf));
    double* d_acc = reinterpret_cast<double*>(jbuf + o_acc);
    HIP_TRY(hipMemcpyAsync(jbuf + o_b, blj.data(), sizeof(BilinJob) * blj.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(d_acc, 0, sizeof(double) * 2 * nacc, st));
    launch_bilinear(reinterpret_cast<BilinJob*>(jbuf + o_b), (int)blj.size(), btiles, d_acc, st);
    HIP_TRY(hipGetLastError());
    std::vector<double> acc(2 * nacc);
    HIP_TRY(hipMemcpyAsync(acc.data(), d_acc, sizeof(double) * acc.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    // ---- the right-hand side f on interface 1 (incident field and its
    //      normal derivative, negated) moves with that interface's nodes:
    //      its term is l_eta^T df = -z_1^T df
    for (int pidx = 0; pidx < np_; ++pidx) {
      const Par& pp = par[p0 + pidx];
      for (int a = 0; a < n_angles; ++a) {
        double dr = acc[2 * ((size_t)a * np_ + pidx)], di = acc[2 * ((size_t)a * np_ + pidx) + 1];
        if (pp.i == 0) {
          const double kx = s->k[0] * std::cos(theta[a]), ky = s->k[0] * std::sin(theta[a]);
          const int N1 = s->N[0];
          double fr = 0.0, fi = 0.0;  // z_1^T (f+ - f-)
          for (int sg = 0; sg < 2; ++sg) {
            const HostCurve& c = cur[2 * pidx + sg];
            const double w = (sg == 0 ? 1.0 : -1.0) * 0.5 / hstep;
            for (int j = 0; j < N1; ++j) {
              const double ang = kx * c.x[j] + ky * (c.y0 + c.y[j]);
              const double cs = std::cos(ang), sn = std::sin(ang);
              const double dn = kx * c.nx[j] + ky * c.ny[j];
              const double f0r = -cs, f0i = -sn;     // -e
              const double f1r = dn * sn, f1i = -dn * cs;  // -(i dn) e
              const double* z = z1.data() + (size_t)2 * s->n[0] * a;
              fr += w * (z[2 * j] * f0r - z[2 * j + 1] * f0i + z[2 * (N1 + j)] * f1r - z[2 * (N1 + j) + 1] * f1i);
              fi += w * (z[2 * j] * f0i + z[2 * j + 1] * f0r + z[2 * (N1 + j)] * f1i + z[2 * (N1 + j) + 1] * f1r);
            }
          }
          dr -= fr;
          di -= fi;
        }
        const double a0r = aU[(size_t)2 * nK * a + 2 * q0[a]], a0i = aU[(size_t)2 * nK * a + 2 * q0[a] + 1];
        grad_shape[pp.out] += 2.0 * (a0r * dr + a0i * di);
      }
    }
  }
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// batches of independent stacks
// ---------------------------------------------------------------------------
struct mlh_batch_s {
  mlh_ctx ctx = nullptr;
  std::vector<mlh_stack_s*> st;
  mlh_tuning tune{300, 3, 16, 1, 8};
  Runner run;
  std::vector<int64_t> out_off;  // first Bragg order of each stack in the concatenated outputs
  int64_t n_orders = 0;
  // merged fill job tables of every stack, and the clock stamps of a solve
  char* dmem = nullptr;
  FillJob* d_fill = nullptr;
  SelfJob* d_self = nullptr;
  AlpertJob* d_alp = nullptr;
  int n_fill = 0, fill_tiles = 0, n_self = 0, self_tiles = 0, n_alp = 0, alp_blocks = 0;
  unsigned long long* d_clock = nullptr;  // [1 + n_stacks]
  int clock_khz = 0;
};

extern "C" mlh_status mlh_batch_create(mlh_ctx ctx, int32_t n_stacks, const mlh_stack* stacks, mlh_batch* out) {
  if (!ctx || !stacks || !out || n_stacks < 1) return fail(MLH_E_INVALID_ARG, "mlh_batch_create: bad arguments");
  for (int i = 0; i < n_stacks; ++i) {
    if (!stacks[i]) return fail(MLH_E_INVALID_ARG, "mlh_batch_create: NULL stack");
    if (stacks[i]->ctx->device != ctx->device)
      return fail(MLH_E_INVALID_ARG, "mlh_batch_create: every stack must live on the context's device");
    for (int j = 0; j < i; ++j)
      if (stacks[j] == stacks[i]) return fail(MLH_E_INVALID_ARG, "mlh_batch_create: a stack appears twice");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<mlh_batch_s> b(new mlh_batch_s());
  b->ctx = ctx;
  b->st.assign(stacks, stacks + n_stacks);
  std::vector<FillJob> fj;
  std::vector<SelfJob> sj;
  std::vector<AlpertJob> aj;
  for (mlh_stack_s* s : b->st) {
    b->out_off.push_back(b->n_orders);
    b->n_orders += s->nK;
    for (FillJob J : s->h_fill) {
      J.tile_begin += b->fill_tiles;
      fj.push_back(J);
    }
    b->fill_tiles += s->fill_tiles;
    for (SelfJob J : s->h_self) {
      J.tile_begin += b->self_tiles;
      sj.push_back(J);
    }
    b->self_tiles += s->self_tiles;
    for (AlpertJob J : s->h_alp) {
      J.block_begin += b->alp_blocks;
      aj.push_back(J);
    }
    b->alp_blocks += s->alp_blocks;
  }
  b->n_fill = (int)fj.size();
  b->n_self = (int)sj.size();
  b->n_alp = (int)aj.size();
  Arena ar;
  const size_t o_f = ar.reserve(sizeof(FillJob) * fj.size()), o_s = ar.reserve(sizeof(SelfJob) * sj.size()),
               o_a = ar.reserve(sizeof(AlpertJob) * aj.size()),
               o_c = ar.reserve(sizeof(unsigned long long) * (size_t)(n_stacks + 1));
  hipError_t e = hipMalloc((void**)&b->dmem, ar.off);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MLH_E_NOMEM : MLH_E_DEVICE, "batch allocation failed");
  b->d_fill = reinterpret_cast<FillJob*>(b->dmem + o_f);
  b->d_self = reinterpret_cast<SelfJob*>(b->dmem + o_s);
  b->d_alp = reinterpret_cast<AlpertJob*>(b->dmem + o_a);
  b->d_clock = reinterpret_cast<unsigned long long*>(b->dmem + o_c);
  mlh_status r = MLH_OK;
  if (hipMemcpy(b->d_fill, fj.data(), sizeof(FillJob) * fj.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_self, sj.data(), sizeof(SelfJob) * sj.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_alp, aj.data(), sizeof(AlpertJob) * aj.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess)
    r = fail(MLH_E_DEVICE, "batch set-up failed");
  if (r != MLH_OK) {
    (void)hipFree(b->dmem);
    return r;
  }
  *out = b.release();
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_destroy(mlh_batch b) {
  if (!b) return MLH_OK;
  (void)hipSetDevice(b->ctx->device);
  if (b->dmem) (void)hipFree(b->dmem);
  b->run.release();
  delete b;
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_solve(mlh_batch b, const double* theta, int32_t refill, int32_t outputs_on_device,
                                      double* aU, double* aD, int32_t* orders, double* flux_err, double* stack_ms) {
  if (!b || !theta || !aU || !aD) return fail(MLH_E_INVALID_ARG, "mlh_batch_solve: bad arguments");
  if (outputs_on_device != 0 && outputs_on_device != 1)
    return fail(MLH_E_INVALID_ARG, "mlh_batch_solve: outputs_on_device must be 0 or 1");
  if (refill != 0 && refill != 1) return fail(MLH_E_INVALID_ARG, "mlh_batch_solve: refill must be 0 or 1");
  const int ns = (int)b->st.size();
  for (int i = 0; i < ns; ++i)
    if (!theta_ok(theta[i])) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  HIP_TRY(hipSetDevice(b->ctx->device));
  hipStream_t st = b->ctx->stream;
  if (refill) {  // every stack's alpha-independent pieces, in three launches
    launch_self(b->d_self, b->n_self, b->self_tiles, kAlpertA, st);
    launch_alpert(b->d_alp, b->n_alp, b->alp_blocks, kAlpertA, st);
    launch_fill(b->d_fill, b->n_fill, b->fill_tiles, st);
    HIP_TRY(hipGetLastError());
  }
  std::vector<SysSpec> sys(ns);
  std::vector<AngleOut> outs(ns);
  for (int i = 0; i < ns; ++i) {
    sys[i] = SysSpec{b->st[i], {i}};
    AngleOut& o = outs[i];
    o.aU = aU + 2 * b->out_off[i];
    o.aD = aD + 2 * b->out_off[i];
    o.orders = orders ? orders + b->out_off[i] : nullptr;
    o.flux = flux_err ? flux_err + i : nullptr;
    o.eta = nullptr;
  }
  SolveOpts opt;
  opt.on_device = outputs_on_device == 1;
  opt.tstamp = b->d_clock;
  std::vector<double> h_flux;
  MLH_TRY(solve_systems(b->run, b->ctx, b->tune, sys, theta, outs, opt, !opt.on_device, h_flux, nullptr));
  if (flux_err && !opt.on_device)
    for (int i = 0; i < ns; ++i) flux_err[i] = h_flux[i];
  if (stack_ms) {
    std::vector<unsigned long long> clk((size_t)ns + 1);
    HIP_TRY(hipMemcpyAsync(clk.data(), b->d_clock, sizeof(unsigned long long) * clk.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < ns; ++i)
      stack_ms[i] = (double)(clk[i + 1] - clk[0]) / (double)b->clock_khz;
  }
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_get_tuning(mlh_batch b, mlh_tuning* out) {
  if (!b || !out) return fail(MLH_E_INVALID_ARG, "mlh_batch_get_tuning: NULL argument");
  *out = b->tune;
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_set_flux_tolerance(mlh_stack s, double tol) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(MLH_E_INVALID_ARG, "flux tolerance must be finite and >= 0");
  s->flux_tol = tol;
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// launch choices and their autotuning
// ---------------------------------------------------------------------------
static bool tuning_valid(const mlh_tuning& t) {
  return t.rhs_in_step_pct >= 0 && t.rhs_in_step_pct <= 1000 && (t.ls_row_blocks == 3 || t.ls_row_blocks == 4) &&
         (t.gje_rhs_cols == 16 || t.gje_rhs_cols == 8) && (t.asm_in_panels == 0 || t.asm_in_panels == 1) &&
         (t.gemm_slab_k == 8 || t.gemm_slab_k == 16);
}

extern "C" mlh_status mlh_stack_get_tuning(mlh_stack s, mlh_tuning* out) {
  if (!s || !out) return fail(MLH_E_INVALID_ARG, "mlh_stack_get_tuning: NULL argument");
  *out = s->tune;
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_set_tuning(mlh_stack s, const mlh_tuning* t) {
  if (!s || !t) return fail(MLH_E_INVALID_ARG, "mlh_stack_set_tuning: NULL argument");
  if (!tuning_valid(*t)) return fail(MLH_E_INVALID_ARG, "mlh_stack_set_tuning: value out of range");
  s->tune = *t;
  return MLH_OK;
}

// One pass of coordinate descent over the fields, each candidate timed as
// whole solve calls (host planning, graph launch and result copy: what a
// caller waits for), fastest of `reps` after one untimed solve that also
// captures the candidate's graph.  `tune` is the live choice the solve
// reads; it ends at the fastest choice, or where it started on an error.
// ---------------------------------------------------------------------------
// launch-choice cache: the choices an autotune picked, keyed by the device's
// architecture name and the size class of the work, so that work of the same
// class takes them without being timed again.  The class: interface count
// (power-of-two bucket), block orders (all up to 576 / up to 608 / above,
// or mixed), least-squares rows (all up to 384 / above / mixed), systems
// solved at once (bucket 1, 2-4, 5-16, 17-64, more).  With MLH_TUNING_CACHE
// naming a file, entries are appended to it and read back by the next process.
// ---------------------------------------------------------------------------
struct SizeClass {
  int interfaces = 0, maxn = 0, minn = 1 << 30, maxrows = 0, minrows = 1 << 30, systems = 0;
  void add_stack(const mlh_stack_s* s) {
    interfaces += s->I;
    for (int i = 0; i < s->I; ++i) {
      maxn = std::max(maxn, s->n[i]);
      minn = std::min(minn, s->n[i]);
    }
    for (int j = 0; j <= s->I; ++j) {
      int m, c, nc;
      layer_dims(s, j, m, c, nc);
      maxrows = std::max(maxrows, m + c);
      minrows = std::min(minrows, m + c);
    }
  }
};

static std::string tuning_key(int device, const SizeClass& c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ' || ch == '\t') ch = '_';
  int ib = 0;
  while ((1 << (ib + 1)) <= c.interfaces) ++ib;
  auto ncls = [](int n) { return gje_step_fits(n) ? 0 : (n <= kRhsMaxN16 ? 1 : 2); };
  const int nlo = ncls(c.minn), nhi = ncls(c.maxn);
  const int rlo = c.minrows > 384, rhi = c.maxrows > 384;
  const int sb = c.systems <= 1 ? 0 : c.systems <= 4 ? 1 : c.systems <= 16 ? 2 : c.systems <= 64 ? 3 : 4;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/I%d/n%d%d/r%d%d/s%d", arch.c_str(), ib, nlo, nhi, rlo, rhi, sb);
  return buf;
}

static std::mutex g_tune_mu;
static std::map<std::string, mlh_tuning> g_tune_cache;
static bool g_tune_loaded = false;

static void tune_cache_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("MLH_TUNING_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512], key[256];
  mlh_tuning t;
  while (std::fgets(line, sizeof line, f))  // one record a line; a line that does not parse is skipped
    if (std::sscanf(line, "%255s %d %d %d %d %d", key, &t.rhs_in_step_pct, &t.ls_row_blocks, &t.gje_rhs_cols,
                    &t.asm_in_panels, &t.gemm_slab_k) == 6 &&
        tuning_valid(t))
      g_tune_cache[key] = t;  // later lines win
  std::fclose(f);
}

static bool tune_cache_find(const std::string& key, mlh_tuning& out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_load_locked();
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  out = it->second;
  return true;
}

static void tune_cache_store(const std::string& key, const mlh_tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_load_locked();
  g_tune_cache[key] = t;
  const char* path = std::getenv("MLH_TUNING_CACHE");
  if (!path || !*path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), t.rhs_in_step_pct, t.ls_row_blocks, t.gje_rhs_cols,
                 t.asm_in_panels, t.gemm_slab_k);
    std::fclose(f);
  }
}

static std::string stack_tuning_key(mlh_stack s, int32_t n_angles, const double* theta) {
  SizeClass c;
  c.add_stack(s);
  std::vector<SysSpec> sys;
  group_by_alpha(s, n_angles, theta, 0, sys);
  c.systems = (int)sys.size();
  return tuning_key(s->ctx->device, c);
}

static std::string batch_tuning_key(mlh_batch b) {
  SizeClass c;
  for (const mlh_stack_s* s : b->st) c.add_stack(s);
  c.systems = (int)b->st.size();
  return tuning_key(b->ctx->device, c);
}

static mlh_status autotune_loop(mlh_tuning& tune, const std::function<mlh_status()>& solve_once, int reps,
                                mlh_tuning* out) {
  const mlh_tuning start = tune;
  auto time_of = [&](const mlh_tuning& t, double& best) -> mlh_status {
    tune = t;
    MLH_TRY(solve_once());
    best = 1e300;
    for (int r = 0; r < reps; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      MLH_TRY(solve_once());
      best = std::min(best, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    }
    return MLH_OK;
  };
  mlh_tuning best_t = start;
  double best = 0;
  mlh_status r = time_of(best_t, best);
  const int pct[] = {0, 100, 150, 200, 300, 500, 1000};
  const int rows[] = {3, 4};
  const int cols[] = {16, 8};
  const int asmp[] = {1, 0};
  const int slabs[] = {8, 16};
  auto sweep = [&](int32_t mlh_tuning::*field, const int* vals, int nv) {
    for (int i = 0; i < nv && r == MLH_OK; ++i) {
      mlh_tuning t = best_t;
      t.*field = vals[i];
      if (t.*field == best_t.*field) continue;
      double ti = 0;
      r = time_of(t, ti);
      if (r == MLH_OK && ti < best) {
        best = ti;
        best_t = t;
      }
    }
  };
  sweep(&mlh_tuning::rhs_in_step_pct, pct, 7);
  sweep(&mlh_tuning::ls_row_blocks, rows, 2);
  sweep(&mlh_tuning::gje_rhs_cols, cols, 2);
  sweep(&mlh_tuning::asm_in_panels, asmp, 2);
  sweep(&mlh_tuning::gemm_slab_k, slabs, 2);
  if (r != MLH_OK) {
    tune = start;
    return r;
  }
  tune = best_t;
  if (out) *out = best_t;
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_autotune(mlh_stack s, int32_t n_angles, const double* theta, int32_t reps,
                                         mlh_tuning* out) {
  if (!s || !theta || n_angles < 1 || reps < 1) return fail(MLH_E_INVALID_ARG, "mlh_stack_autotune: bad arguments");
  for (int a = 0; a < n_angles; ++a)
    if (!theta_ok(theta[a])) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  const size_t nc = (size_t)2 * s->nK * n_angles;
  std::vector<double> aU(nc), aD(nc);
  MLH_TRY(autotune_loop(
      s->tune,
      [&]() { return solve_impl(s, n_angles, theta, aU.data(), aD.data(), nullptr, nullptr, nullptr, false, SolveOpts()); },
      reps, out));
  tune_cache_store(stack_tuning_key(s, n_angles, theta), s->tune);
  return MLH_OK;
}

extern "C" mlh_status mlh_stack_tune_cached(mlh_stack s, int32_t n_angles, const double* theta, mlh_tuning* out,
                                            int32_t* found) {
  if (!s || !theta || n_angles < 1 || !found) return fail(MLH_E_INVALID_ARG, "mlh_stack_tune_cached: bad arguments");
  for (int a = 0; a < n_angles; ++a)
    if (!theta_ok(theta[a])) return fail(MLH_E_INVALID_ARG, "incident angle must lie in (-pi, 0)");
  mlh_tuning t;
  *found = tune_cache_find(stack_tuning_key(s, n_angles, theta), t) ? 1 : 0;
  if (*found) s->tune = t;
  if (out) *out = s->tune;
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_set_tuning(mlh_batch b, const mlh_tuning* t) {
  if (!b || !t) return fail(MLH_E_INVALID_ARG, "mlh_batch_set_tuning: NULL argument");
  if (!tuning_valid(*t)) return fail(MLH_E_INVALID_ARG, "mlh_batch_set_tuning: value out of range");
  b->tune = *t;
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_autotune(mlh_batch b, const double* theta, int32_t reps, mlh_tuning* out) {
  if (!b || !theta || reps < 1) return fail(MLH_E_INVALID_ARG, "mlh_batch_autotune: bad arguments");
  std::vector<double> aU((size_t)2 * b->n_orders), aD((size_t)2 * b->n_orders);
  MLH_TRY(autotune_loop(
      b->tune, [&]() { return mlh_batch_solve(b, theta, 0, 0, aU.data(), aD.data(), nullptr, nullptr, nullptr); },
      reps, out));
  tune_cache_store(batch_tuning_key(b), b->tune);
  return MLH_OK;
}

extern "C" mlh_status mlh_batch_tune_cached(mlh_batch b, mlh_tuning* out, int32_t* found) {
  if (!b || !found) return fail(MLH_E_INVALID_ARG, "mlh_batch_tune_cached: bad arguments");
  mlh_tuning t;
  *found = tune_cache_find(batch_tuning_key(b), t) ? 1 : 0;
  if (*found) b->tune = t;
  if (out) *out = b->tune;
  return MLH_OK;
}

// ---------------------------------------------------------------------------
// inspection entry points
// ---------------------------------------------------------------------------
extern "C" mlh_status mlh_debug_get_piece(mlh_stack s, int32_t which, int32_t index, int32_t piece, double* out,
                                          int32_t* rows, int32_t* cols) {
  if (!s) return fail(MLH_E_INVALID_ARG, "NULL stack");
  const int I = s->I;
  int r = 0, c = 0, np = 1;
  const cplx* base = nullptr;
  auto need = [&](bool ok) { return ok; };
  switch (which) {
    case 0:
      if (!need(index >= 0 && index < I)) break;
      r = c = s->n[index];
      np = 3;
      base = s->A_self[index];
      break;
    case 1:
    case 2:
      if (!need(index >= 0 && index + 1 < I)) break;
      r = which == 1 ? s->n[index] : s->n[index + 1];
      c = which == 1 ? s->n[index + 1] : s->n[index];
      np = 3;
      base = which == 1 ? s->A_up[index] : s->A_dn[index];
      break;
    case 3:
    case 4:
      if (!need(index >= 0 && index < I)) break;
      r = s->n[index];
      c = s->P;
      base = which == 3 ? s->B_own[index] : s->B_below[index];
      break;
    case 5:
      if (!need(index >= 0 && index < I)) break;
      r = 2 * s->Mw;
      c = s->n[index];
      np = 2;
      base = s->C_own[index];
      break;
    case 6:
      if (!need(index >= 1 && index <= I)) break;
      r = 2 * s->Mw;
      c = s->n[index - 1];
      np = 2;
      base = s->C_above[index];
      break;
    case 7:
      if (!need(index >= 0 && index <= I)) break;
      r = 2 * s->Mw;
      c = s->P;
      np = 2;
      base = s->Q[index];
      break;
    case 8:
    case 9:
      r = 2 * s->Mud;
      c = which == 8 ? s->n[0] : s->n[I - 1];
      np = 3;
      base = which == 8 ? s->Z_U : s->Z_D;
      break;
    case 10:
    case 11:
      r = 2 * s->Mud;
      c = s->P;
      base = which == 10 ? s->V_U : s->V_D;
      break;
    default:
      break;
  }
  if (!base || piece < 0 || piece >= np) return fail(MLH_E_INVALID_ARG, "mlh_debug_get_piece: no such piece");
  if (rows) *rows = r;
  if (cols) *cols = c;
  if (out) {
    HIP_TRY(hipSetDevice(s->ctx->device));
    HIP_TRY(hipStreamSynchronize(s->ctx->stream));
    HIP_TRY(hipMemcpy(out, base + (size_t)piece * r * c, cbytes((size_t)r * c), hipMemcpyDeviceToHost));
  }
  return MLH_OK;
}

extern "C" mlh_status mlh_debug_hankel(mlh_ctx ctx, int32_t n, const double* x, double* out) {
  if (!ctx || n < 0 || (n > 0 && (!x || !out))) return fail(MLH_E_INVALID_ARG, "mlh_debug_hankel: bad arguments");
  for (int i = 0; i < n; ++i)
    if (!(x[i] > 0)) return fail(MLH_E_INVALID_ARG, "mlh_debug_hankel: arguments must be positive");
  if (n == 0) return MLH_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  double* d = nullptr;
  HIP_TRY(hipMalloc((void**)&d, sizeof(double) * 5 * n));
  hipError_t e = hipMemcpy(d, x, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_hankel_eval(d, d + n, n, ctx->stream);
    e = hipStreamSynchronize(ctx->stream);
  }
  if (e == hipSuccess) e = hipMemcpy(out, d + n, sizeof(double) * 4 * n, hipMemcpyDeviceToHost);
  const hipError_t fe = hipFree(d);
  if (e == hipSuccess) e = fe;
  if (e != hipSuccess) return fail(MLH_E_DEVICE, hipGetErrorString(e));
  return MLH_OK;
}

extern "C" mlh_status mlh_debug_zgemm(mlh_ctx ctx, int32_t m, int32_t n, int32_t k, const double* alpha,
                                      const double* A, const double* Bm, double* C) {
  if (!ctx || m < 1 || n < 1 || k < 1 || !alpha || !A || !Bm || !C)
    return fail(MLH_E_INVALID_ARG, "mlh_debug_zgemm: bad arguments");
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t na = (size_t)m * k, nb = (size_t)k * n, nc = (size_t)m * n;
  char* d = nullptr;
  const size_t bytes = cbytes(na + nb + nc) + sizeof(GemmDesc) + 256;
  HIP_TRY(hipMalloc((void**)&d, bytes));
  cplx* dA = reinterpret_cast<cplx*>(d);
  cplx* dB = dA + na;
  cplx* dC = dB + nb;
  GemmDesc* dg = reinterpret_cast<GemmDesc*>(d + ((cbytes(na + nb + nc) + 255) & ~size_t(255)));
  GemmDesc G{};
  G.A = dA;
  G.B = dB;
  G.C = dC;
  G.alpha = cx(alpha[0], alpha[1]);
  G.k2 = 0;
  G.C0 = dC;
  G.ldc0 = m;
  G.m = m;
  G.n = n;
  G.k = k;
  G.lda = m;
  G.ldb = k;
  G.ldc = m;
  G.tiles_m = (m + kGemmTile - 1) / kGemmTile;
  G.tile_begin = 0;
  const int tiles = G.tiles_m * ((n + kGemmTile - 1) / kGemmTile);
  hipError_t e = hipMemcpy(dA, A, cbytes(na), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dB, Bm, cbytes(nb), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dC, C, cbytes(nc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dg, &G, sizeof(G), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_gemm(dg, 1, tiles, ctx->stream);
    e = hipStreamSynchronize(ctx->stream);
  }
  if (e == hipSuccess) e = hipMemcpy(C, dC, cbytes(nc), hipMemcpyDeviceToHost);
  const hipError_t fe = hipFree(d);
  if (e == hipSuccess) e = fe;
  if (e != hipSuccess) return fail(MLH_E_DEVICE, hipGetErrorString(e));
  return MLH_OK;
}

extern "C" mlh_status mlh_debug_solve_partial(mlh_stack s, double theta, int32_t stop_phase) {
  if (stop_phase < 1 || stop_phase > 4) return fail(MLH_E_INVALID_ARG, "stop_phase must be 1..4");
  double aU[2 * 512], aD[2 * 512], fl[1];
  int ord[512];
  if (!s || 2 * s->K + 1 > 512) return fail(MLH_E_INVALID_ARG, "bad stack");
  SolveOpts o;
  o.stop_phase = stop_phase;
  return solve_impl(s, 1, &theta, aU, aD, ord, fl, nullptr, false, o);
}

extern "C" mlh_status mlh_debug_get_work(mlh_stack s, int32_t which, int32_t index, double* out, int32_t* rows,
                                         int32_t* cols) {
  if (!s || s->dbg_R.empty()) return fail(MLH_E_INVALID_ARG, "no inspection solve has run");
  const int I = s->I;
  // level-0 row block of interface i: [A'_ii | A'_{i,i-1} | A'_{i,i+1} | f~_i]
  auto nl = [&](int i) { return i > 0 ? s->n[i - 1] : 0; };
  auto nu = [&](int i) { return i + 1 < I ? s->n[i + 1] : 0; };
  int r = 0, c1 = 0, c2 = 0;
  const cplx* p1 = nullptr;
  const cplx* p2 = nullptr;
  if (which == 0 && index >= 0 && index < I) {  // [A'_ii | f~_i]
    r = s->n[index];
    c1 = r;
    p1 = s->dbg_R[index];
    c2 = 1;
    p2 = s->dbg_R[index] + (size_t)r * (r + nl(index) + nu(index));
  } else if (which == 1 && index >= 0 && index + 1 < I) {  // A'_{i,i+1}
    r = s->n[index];
    c1 = s->n[index + 1];
    p1 = s->dbg_R[index] + (size_t)r * (r + nl(index));
  } else if (which == 2 && index >= 0 && index + 1 < I) {  // A'_{i+1,i}
    r = s->n[index + 1];
    c1 = s->n[index];
    p1 = s->dbg_R[index + 1] + (size_t)r * r;
  } else if ((which == 3 || which == 4) && index >= 0 && index <= I) {
    int m, cc, nc;
    layer_dims(s, index, m, cc, nc);
    r = m + cc;
    c1 = which == 3 ? cc : nc;
    p1 = which == 3 ? s->dbg_S[index] : s->dbg_RHS[index];
  } else if (which == 6 && index >= 0 && index < I) {
    r = s->n[index];
    c1 = 1;
    p1 = s->dbg_eta[index];
  }
  if (!p1) return fail(MLH_E_INVALID_ARG, "mlh_debug_get_work: no such block");
  if (rows) *rows = r;
  if (cols) *cols = c1 + c2;
  if (out) {
    HIP_TRY(hipSetDevice(s->ctx->device));
    HIP_TRY(hipMemcpy(out, p1, cbytes((size_t)r * c1), hipMemcpyDeviceToHost));
    if (p2) HIP_TRY(hipMemcpy(out + (size_t)2 * r * c1, p2, cbytes((size_t)r * c2), hipMemcpyDeviceToHost));
  }
  return MLH_OK;
}

extern "C" mlh_status mlh_profile_step(mlh_stack s, double theta, mlh_profile* out) {
  return mlh_profile_solve(s, 1, &theta, out);
}

extern "C" mlh_status mlh_profile_solve(mlh_stack s, int32_t n_angles, const double* theta, mlh_profile* out) {
  if (!s || !out || !theta || n_angles < 1) return fail(MLH_E_INVALID_ARG, "mlh_profile_solve: bad arguments");
  std::memset(out, 0, sizeof(*out));
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  EvTimer T{st};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, st));
  T.begin(&out->fill_self_ms);
  launch_self(s->d_self, s->n_self, s->self_tiles, kAlpertA, st);
  T.end();
  T.begin(&out->fill_alpert_ms);
  launch_alpert(s->d_alp, s->n_alp, s->alp_blocks, kAlpertA, st);
  T.end();
  T.begin(&out->fill_pairs_ms);
  launch_fill(s->d_fill, s->n_fill, s->fill_tiles, st);
  T.end();
  HIP_TRY(hipGetLastError());
  HIP_TRY(T.collect());
  const int nK = 2 * s->K + 1;
  std::vector<double> aU((size_t)2 * nK * n_angles), aD((size_t)2 * nK * n_angles);
  std::vector<int> ord((size_t)nK * n_angles);
  std::vector<double> fl(n_angles);
  SolveOpts o;
  o.prof = out;
  mlh_status r = solve_impl(s, n_angles, theta, aU.data(), aD.data(), ord.data(), fl.data(), nullptr, false, o);
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  hipError_t te = hipEventElapsedTime(&ms, e0, e1);
  out->total_ms = ms;
  const hipError_t d0 = hipEventDestroy(e0), d1 = hipEventDestroy(e1);
  if (r != MLH_OK) return r;
  if (te == hipSuccess) te = d0 != hipSuccess ? d0 : d1;
  HIP_TRY(te);
  return r;
}
