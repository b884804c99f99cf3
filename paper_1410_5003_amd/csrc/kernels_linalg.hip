// Dense complex float64 linear algebra of the solve phase (Sec. 3):
//
//  zgemm_kernel     batched C = C0 + alpha (A B + A2 B2) on the FP64 matrix
//                   cores (v_mfma_f64_16x16x4f64, three real products per
//                   complex product); Schur updates eq. (74)-(78) and the
//                   sweep update.
//                   Operand layout of the 16x16x4 f64 instruction: lane l holds
//                   A[l%16][l/16] and B[l/16][l%16]; accumulator register r of
//                   lane l holds D[l/16 + 4r][l%16].
//  rb_setup_kernel  Rayleigh-Bloch rows W_U, W_D (eq. (59)) and the
//                   incident-field right-hand side f (Sec. 2.2).
//  bragg_kernel     a^U = -[X_1 eta_1]_a, a^D = -[X_{I+1} eta_I]_a (Sec. 3.3)
//                   and the flux error eq. (86).
#include <algorithm>

#include "internal.hpp"

namespace mlh {

typedef double dvec4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ inline int find_tile(const T* d, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_begin <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline double2 ld2(const cplx* p) { return ldc(p); }
__device__ inline void st2(cplx* p, double re, double im) {
  stc(p, re, im);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// batched complex GEMM C = C0 + alpha (A B + A2 B2): one workgroup of four
// wavefronts per kGemmTile x kGemmTile tile of C, each wavefront a 32 x 32
// quarter as 2 x 2 blocks of 16 x 16 on the FP64 matrix cores.  K runs in
// slabs of 8 or 16 in two LDS buffers; the next slab goes from global memory
// straight into the other buffer while the current one is multiplied (one
// barrier per slab).  A complex product takes three real ones
// (T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi); re = T1 - T2,
// im = T3 - T1 - T2), a quarter fewer matrix-core operations than four.
// ---------------------------------------------------------------------------
static_assert(kGemmTile == 64, "slab loads: one A instruction per k of 64 rows");

// The slab buffers, two of each, kGK deep (8 or 16: a launch choice),
// filled straight from global memory by 16-byte global-to-LDS loads (lane i
// of an instruction lands at base + 16 i), so the next slab needs no staging
// registers: A as [k][row] (one instruction per k: 64 consecutive rows), B
// as [col][k ^ (col mod kGK)] (one instruction per 64 / kGK columns x kGK
// k, each column's slab read in one piece; the XOR puts the operand reads
// of consecutive columns on distinct banks).
template <int kGK>
using SlabA = double2[kGK][kGemmTile];
template <int kGK>
using SlabB = double2[kGemmTile][kGK];
typedef const void __attribute__((address_space(1)))* gvoid_p;
typedef void __attribute__((address_space(3)))* lvoid_p;
__device__ __forceinline__ void lds_load16(const cplx* src, double2* lds_base) {
  __builtin_amdgcn_global_load_lds((gvoid_p)src, (lvoid_p)lds_base, 16, 0, 0);
}

// One tile.  kFull: the tile lies wholly inside C, so no 16 x 16 block is
// skipped and the k-steps of a slab have no branch between their products;
// edge tiles take the checked form.
template <bool kFull, int kGK>
__device__ __forceinline__ void zgemm_tile(const GemmDesc& G, int row0, int col0, SlabA<kGK>& a0, SlabB<kGK>& b0,
                                           SlabA<kGK>& a1, SlabB<kGK>& b1) {
  static_assert(kGK == 8 || kGK == 16, "slab depth");
  constexpr int kBCols = kGemmTile / kGK;  // B columns per load instruction
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int m = G.m, n = G.n, K1 = G.k, K = G.k + G.k2;
  // 16 x 16 blocks of the wave that hold rows / columns of C (the ragged
  // edge tiles and the narrow right-hand-side products leave the others out)
  const bool rin[2] = {kFull || row0 + wm < m, kFull || row0 + wm + 16 < m};
  const bool cin[2] = {kFull || col0 + wn < n, kFull || col0 + wn + 16 < n};
  dvec4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      t1[b][c] = dvec4{0, 0, 0, 0};
      t2[b][c] = dvec4{0, 0, 0, 0};
      t3[b][c] = dvec4{0, 0, 0, 0};
    }
  const cplx* const A1 = G.A;
  const cplx* const A2 = G.A2;
  const cplx* const B1 = G.B;
  const cplx* const B2 = G.B2;
  const int lda = G.lda, lda2 = G.lda2, ldb = G.ldb, ldb2 = G.ldb2;
  // Slab k0 into (Sa, Sb): wave w loads A's k rows w, w + 4, ... and B's
  // columns 16 w .. 16 w + 15.  Indices are clamped: rows of A past m and
  // columns of B past n only reach entries of C that are not stored, and k
  // past K is zeroed in A once the slab has landed.
  const int arow = min(row0 + lane, m - 1);
  auto issue = [&](int k0, SlabA<kGK>& Sa, SlabB<kGK>& Sb) {
#pragma unroll
    for (int h = 0; h < kGK / 4; ++h) {
      const int kl = wave + 4 * h;
      const int kc = min(k0 + kl, K - 1);
      const cplx* src = kc < K1 ? A1 + (size_t)kc * lda + arow : A2 + (size_t)(kc - K1) * lda2 + arow;
      lds_load16(src, &Sa[kl][0]);
    }
#pragma unroll
    for (int h = 0; h < kGK / 4; ++h) {
      const int cl = 16 * wave + kBCols * h + lane / kGK;
      const int kk = (lane % kGK) ^ (cl % kGK);
      const int cc = min(col0 + cl, n - 1), kc = min(k0 + kk, K - 1);
      const cplx* src = kc < K1 ? B1 + (size_t)cc * ldb + kc : B2 + (size_t)cc * ldb2 + (kc - K1);
      lds_load16(src, &Sb[16 * wave + kBCols * h][0]);
    }
  };
  auto slab = [&](const SlabA<kGK>& Sa, const SlabB<kGK>& Sb) {
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      const int ka = ks + lq;
      double ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double2 va = Sa[ka][wm + 16 * b + lr];
        const int col = wn + 16 * b + lr;
        const double2 vb = Sb[col][ka ^ (col % kGK)];
        ar[b] = va.x;
        ai[b] = va.y;
        as[b] = va.x + va.y;
        br[b] = vb.x;
        bi[b] = vb.y;
        bs[b] = vb.x + vb.y;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (!kFull && !(rin[b] && cin[c])) continue;
          t1[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[b], br[c], t1[b][c], 0, 0, 0);
          t2[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[b], bi[c], t2[b][c], 0, 0, 0);
          t3[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[b], bs[c], t3[b][c], 0, 0, 0);
        }
    }
  };
  // slab k0 has landed in (Sa, Sb): zero A's k past K on the last slab,
  // start the next slab's loads into (Na, Nb), multiply
  auto step = [&](int k0, SlabA<kGK>& Sa, SlabB<kGK>& Sb, SlabA<kGK>& Na, SlabB<kGK>& Nb) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the slab have landed
    __syncthreads();                // every wave's have; every wave is done with (Na, Nb)
    if (k0 + kGK > K) {             // uniform over the workgroup
      for (int e = tid; e < kGK * kGemmTile; e += 256)
        if (k0 + e / kGemmTile >= K) Sa[e / kGemmTile][e % kGemmTile] = make_double2(0.0, 0.0);
      __syncthreads();
    }
    if (k0 + kGK < K) issue(k0 + kGK, Na, Nb);
    slab(Sa, Sb);
  };
  // slabs in pairs, so that each buffer is a named array at every use (no
  // select between the two for the loads' destinations or the reads)
  if (K > 0) issue(0, a0, b0);
  for (int k0 = 0; k0 < K; k0 += 2 * kGK) {
    step(k0, a0, b0, a1, b1);
    if (k0 + kGK >= K) break;
    step(k0 + kGK, a1, b1, a0, b0);
  }
  // C0 first, every load in flight at once (clamped addresses), then C
  const cplx* const C0 = G.C0;
  cplx* const Cm = G.C;
  const int ldc = G.ldc, ldc0 = G.ldc0;
  const double alr = G.alpha.re, ali = G.alpha.im;
  double2 c0v[2][2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = min(col0 + wn + 16 * c + lr, n - 1), row = min(row0 + wm + 16 * b + lq + 4 * r, m - 1);
        c0v[c][b][r] = C0 ? ld2(C0 + (size_t)col * ldc0 + row) : make_double2(0.0, 0.0);
      }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = col0 + wn + 16 * c + lr;
    if (!kFull && col >= n) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm + 16 * b + lq + 4 * r;
        if (kFull || row < m) {
          const double xr = t1[b][c][r] - t2[b][c][r], xi = t3[b][c][r] - t1[b][c][r] - t2[b][c][r];
          const double2 cv = c0v[c][b][r];
          st2(Cm + (size_t)col * ldc + row, cv.x + alr * xr - ali * xi, cv.y + alr * xi + ali * xr);
        }
      }
  }
}

template <int kGK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void zgemm_kernel(const GemmDesc* __restrict__ descs, int ndesc, int tile0) {
  const int tile = tile0 + (int)blockIdx.x;
  const GemmDesc& G = descs[find_tile(descs, ndesc, tile)];
  const int lt = tile - G.tile_begin;
  const int row0 = (lt % G.tiles_m) * kGemmTile, col0 = (lt / G.tiles_m) * kGemmTile;
  __shared__ SlabA<kGK> a0, a1;
  __shared__ SlabB<kGK> b0, b1;
  if (row0 + kGemmTile <= G.m && col0 + kGemmTile <= G.n)  // uniform over the workgroup
    zgemm_tile<true, kGK>(G, row0, col0, a0, b0, a1, b1);
  else
    zgemm_tile<false, kGK>(G, row0, col0, a0, b0, a1, b1);
}

// ---------------------------------------------------------------------------
// least squares of one layer: Householder QR of S = [Q; mu I]
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Rayleigh-Bloch orders, W blocks and the incident right-hand side
// ---------------------------------------------------------------------------
__device__ inline int rb_n0(double kappa0, double d) { return (int)floor(-kappa0 * d / (2.0 * kPi) + 0.5); }

__device__ inline cplx vert_wavenumber(double k, double kappa) {
  const double q = k * k - kappa * kappa;
  if (fabs(q) <= 1e-14 * k * k) return {0.0, 0.0};
  if (q > 0) return {sqrt(q), 0.0};
  return {0.0, sqrt(-q)};
}

__global__ __launch_bounds__(256) void rb_setup_kernel(const AngleDesc* __restrict__ ang) {
  const AngleDesc& A = ang[blockIdx.x];
  const StackConsts& sc = A.sc;
  const int nK = 2 * sc.K + 1;
  const double kappa0 = sc.k1 * cos(A.theta);
  const int n0 = rb_n0(kappa0, sc.d);
  const int tid = threadIdx.x;
  const int r0 = 2 * sc.Mw;
  for (int e = tid; A.owner && e < sc.Mud * nK; e += 256) {  // W rows: once per system
    const int mrow = e % sc.Mud, q = e / sc.Mud;
    const double kap = kappa0 + 2.0 * kPi * (double)(n0 - sc.K + q) / sc.d;
    double s, c;
    sincos(kap * sc.xud[mrow], &s, &c);
    const cplx ku = vert_wavenumber(sc.k1, kap), kd = vert_wavenumber(sc.kI1, kap);
    cplx* wu = A.S0 + (size_t)(sc.P + q) * A.ldS0 + r0;
    cplx* wd = A.SI + (size_t)(sc.P + q) * A.ldSI + r0;
    st2(wu + mrow, -c, -s);
    st2(wd + mrow, -c, -s);
    // -i k^U e  and  +i k^D e
    const cplx iku = {-ku.im, ku.re}, ikd = {-kd.im, kd.re};
    st2(wu + sc.Mud + mrow, -(iku.re * c - iku.im * s), -(iku.re * s + iku.im * c));
    st2(wd + sc.Mud + mrow, (ikd.re * c - ikd.im * s), (ikd.re * s + ikd.im * c));
  }
  const double kx = sc.k1 * cos(A.theta), ky = sc.k1 * sin(A.theta);
  for (int j = tid; j < sc.N1; j += 256) {
    double s, c;
    sincos(kx * sc.x1[j] + ky * (sc.y0_1 + sc.y1[j]), &s, &c);
    const double dn = kx * sc.nx1[j] + ky * sc.ny1[j];
    st2(A.F0 + j, -c, -s);
    // -(i dn) e
    st2(A.F0 + sc.N1 + j, dn * s, -dn * c);
  }
}

// one workgroup per angle: lane q of every wave takes order q, the 8 waves
// split the density index and their partial sums meet in LDS
__global__ __launch_bounds__(512) void bragg_kernel(const AngleDesc* __restrict__ ang) {
  const AngleDesc& A = ang[blockIdx.x];
  const StackConsts& sc = A.sc;
  const int nK = 2 * sc.K + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double kappa0 = sc.k1 * cos(A.theta);
  const int n0 = rb_n0(kappa0, sc.d);
  const int n1 = 2 * sc.N1, nI = 2 * sc.NI;
  __shared__ double2 pu[8][64], pd[8][64];
  double fl = 0.0;
  for (int q0 = 0; q0 < nK; q0 += 64) {
    const int q = q0 + lane;
    double ur = 0.0, ui = 0.0, dr = 0.0, di = 0.0;
    // eight columns in flight per lane (clamped indices; lanes past nK
    // compute a copy of the last order and store nothing)
    const int qc = min(q, nK - 1);
    constexpr int kU = 8;
    for (int j0 = wave; j0 < n1; j0 += 8 * kU) {
      double2 x[kU], e[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = min(j0 + 8 * u, n1 - 1);
        x[u] = ld2(A.X0 + (size_t)j * A.ldX0 + sc.P + qc);
        e[u] = ld2(A.eta0 + j);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const bool in = j0 + 8 * u < n1;
        ur -= in ? x[u].x * e[u].x - x[u].y * e[u].y : 0.0;
        ui -= in ? x[u].x * e[u].y + x[u].y * e[u].x : 0.0;
      }
    }
    for (int j0 = wave; j0 < nI; j0 += 8 * kU) {
      double2 x[kU], e[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = min(j0 + 8 * u, nI - 1);
        x[u] = ld2(A.XI + (size_t)j * A.ldXI + sc.P + qc);
        e[u] = ld2(A.etaI + j);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const bool in = j0 + 8 * u < nI;
        dr -= in ? x[u].x * e[u].x - x[u].y * e[u].y : 0.0;
        di -= in ? x[u].x * e[u].y + x[u].y * e[u].x : 0.0;
      }
    }
    pu[wave][lane] = make_double2(ur, ui);
    pd[wave][lane] = make_double2(dr, di);
    __syncthreads();
    if (wave == 0 && q < nK) {
      ur = ui = dr = di = 0.0;
      for (int w = 0; w < 8; ++w) {
        ur += pu[w][lane].x;
        ui += pu[w][lane].y;
        dr += pd[w][lane].x;
        di += pd[w][lane].y;
      }
      st2(A.aU + q, ur, ui);
      st2(A.aD + q, dr, di);
      A.orders[q] = n0 - sc.K + q;
      const double kap = kappa0 + 2.0 * kPi * (double)(n0 - sc.K + q) / sc.d;
      const cplx ku = vert_wavenumber(sc.k1, kap), kd = vert_wavenumber(sc.kI1, kap);
      if (ku.im == 0.0 && ku.re > 0.0) fl += ku.re * (ur * ur + ui * ui);
      if (kd.im == 0.0 && kd.re > 0.0) fl += kd.re * (dr * dr + di * di);
    }
    __syncthreads();
  }
  if (wave == 0) {
    fl = wave_sum(fl);
    if (lane == 0) {
      const double inc = sc.k1 * fabs(sin(A.theta));
      A.flux[0] = (fl - inc) / inc;
      if (A.tdone) A.tdone[0] = (unsigned long long)wall_clock64();
    }
  }
}

void launch_gemm(const GemmDesc* d_desc, int ndesc, int total_tiles, hipStream_t st, int slab_k) {
  for (int t0 = 0; t0 < total_tiles; t0 += kMaxLaunchBlocks) {
    const dim3 grid(std::min(kMaxLaunchBlocks, total_tiles - t0));
    if (slab_k == 16)
      hipLaunchKernelGGL(zgemm_kernel<16>, grid, dim3(256), 0, st, d_desc, ndesc, t0);
    else
      hipLaunchKernelGGL(zgemm_kernel<8>, grid, dim3(256), 0, st, d_desc, ndesc, t0);
  }
}
__global__ void stamp_kernel(unsigned long long* p) {
  if (threadIdx.x == 0) p[0] = (unsigned long long)wall_clock64();
}

void launch_stamp(unsigned long long* p, hipStream_t st) { hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, p); }

void launch_rb_setup(const AngleDesc* d_ang, int nang, hipStream_t st) {
  if (nang > 0) hipLaunchKernelGGL(rb_setup_kernel, dim3(nang), dim3(256), 0, st, d_ang);
}
void launch_bragg(const AngleDesc* d_ang, int nang, hipStream_t st) {
  if (nang > 0) hipLaunchKernelGGL(bragg_kernel, dim3(nang), dim3(512), 0, st, d_ang);
}

}  // namespace mlh
