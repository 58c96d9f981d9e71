// Workgroup-level dense linear algebra for the boundary-MPS evaluation.
//
// Every routine is executed by all threads of one workgroup together; `tid`
// and `nt` are the thread index and the workgroup size.  Operands live in LDS
// or in global memory (generic pointers).  Callers place __syncthreads()
// between dependent calls; each routine starts reading only what the caller
// has made visible and ends with a barrier when it leaves shared results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pg {

// Linear index i -> (i % n0) * s0 + (i / n0) * s1: one GEMM dimension that
// runs over two tensor legs with independent strides.
// q = i / n and r = i % n from a float reciprocal inv ~ 1/n: the truncated
// estimate is off by at most one either way, and one correction step makes it
// exact for 0 <= i < 2^20, 1 <= n <= 4096 (also when inv is 1 ulp off).  An
// integer division by a run-time value costs tens of instructions.
__host__ __device__ inline int qdiv(int i, int n, float inv, int& r) {
  int q = (int)((float)i * inv);
  r = i - q * n;
  if (r >= n) {
    ++q;
    r -= n;
  } else if (r < 0) {
    --q;
    r += n;
  }
  return q;
}

struct Map {
  int n0, s0, s1;
  float inv;  // 1 / n0
};
__host__ __device__ inline Map map1(int s) { return Map{1 << 30, s, 0, 0x1p-30f}; }
__host__ __device__ inline Map map2(int n0, int s0, int s1) {
  return Map{n0, s0, s1, 1.0f / (float)n0};
}
__device__ inline int mapoff(const Map& m, int i) {
  int r;
  const int q = qdiv(i, m.n0, m.inv, r);
  return r * m.s0 + q * m.s1;
}

// C(m, n) = alpha * sum_k A(m, k) B(k, n)  (+ C(m, n) when acc).
// K = K0 * K1 with k = k1 * K0 + k0; A(m,k) at A[mapoff(am,m) + k0*ak0 + k1*ak1],
// B(k,n) at B[k0*bk0 + k1*bk1 + mapoff(bn,n)], C at C[mapoff(cm,m) + mapoff(cn,n)].
struct Gemm {
  int Md, Nd, K0, K1;
  const double* A;
  Map am;
  int ak0, ak1;
  const double* B;
  Map bn;
  int bk0, bk1;
  double* C;
  Map cm, cn;
  double alpha;
  int acc;
};

template <int TM, int TN>
__device__ void gemm_tiles(const Gemm& g, int tid, int nt) {
  const int tm = (g.Md + TM - 1) / TM, tn = (g.Nd + TN - 1) / TN;
  const float itn = 1.0f / (float)tn;
  for (int t = tid; t < tm * tn; t += nt) {
    int ni;
    const int mi = qdiv(t, tn, itn, ni);
    int aoff[TM], cmo[TM], boff[TN], cno[TN];
#pragma unroll
    for (int r = 0; r < TM; ++r) {
      int m = mi * TM + r;
      m = m < g.Md ? m : g.Md - 1;
      aoff[r] = mapoff(g.am, m);
      cmo[r] = mapoff(g.cm, m);
    }
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      int n = ni * TN + c;
      n = n < g.Nd ? n : g.Nd - 1;
      boff[c] = mapoff(g.bn, n);
      cno[c] = mapoff(g.cn, n);
    }
    double acc[TM][TN];
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
      for (int c = 0; c < TN; ++c) acc[r][c] = 0.0;
    for (int k1 = 0; k1 < g.K1; ++k1) {
      const double* Ap = g.A + (int64_t)k1 * g.ak1;
      const double* Bp = g.B + (int64_t)k1 * g.bk1;
      for (int k0 = 0; k0 < g.K0; ++k0) {
        double a[TM], b[TN];
#pragma unroll
        for (int r = 0; r < TM; ++r) a[r] = Ap[aoff[r] + k0 * g.ak0];
#pragma unroll
        for (int c = 0; c < TN; ++c) b[c] = Bp[boff[c] + k0 * g.bk0];
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
          for (int c = 0; c < TN; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
      }
    }
#pragma unroll
    for (int r = 0; r < TM; ++r) {
      if (mi * TM + r >= g.Md) continue;
#pragma unroll
      for (int c = 0; c < TN; ++c) {
        if (ni * TN + c >= g.Nd) continue;
        double* p = g.C + cmo[r] + cno[c];
        double v = g.alpha * acc[r][c];
        *p = g.acc ? *p + v : v;
      }
    }
  }
}

// Tile shape picked from the problem shape: thin problems use thin tiles, and
// small outputs use small tiles so that most threads get work.
__device__ inline void gemm(const Gemm& g, int tid, int nt) {
  if (g.Md <= 0 || g.Nd <= 0) return;
  const int outs = g.Md * g.Nd;
  if (g.Nd <= 2)
    gemm_tiles<4, 1>(g, tid, nt);
  else if (g.Md <= 2)
    gemm_tiles<1, 4>(g, tid, nt);
  else if (outs >= 8 * nt)
    gemm_tiles<4, 4>(g, tid, nt);
  else
    gemm_tiles<2, 2>(g, tid, nt);
}

// ---------------------------------------------------------------------------
// Matrix-core GEMM, float64: C(m, n) = alpha * sum_k A(m, k) B(k, n) with
// A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] and C placed by maps.
// Each wave owns 16x16 output tiles and walks K four at a time with
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// holds D[4i + l/16][l%16] in accumulator element i.  Out-of-range rows,
// columns and k are fed as zeros, so every lane of the wave issues every MFMA.
// ---------------------------------------------------------------------------
typedef double pg_d4 __attribute__((ext_vector_type(4)));

// rot: tile t goes to wave (t + rot) % (waves), so back-to-back calls
// without a barrier between them spread their tiles over all waves.
__device__ inline void mgemm64(int Md, int Nd, int K, const double* A, int sam, int sak,
                               const double* B, int sbk, int sbn, double* C, Map cm, Map cn,
                               double alpha, int tid, int nt, int rot = 0) {
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int tm = (Md + 15) >> 4, tn = (Nd + 15) >> 4;
  const float itn = 1.0f / (float)tn;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = (wave + nw - rot % nw) % nw; t < tm * tn; t += nw) {
    int ti;
    const int m0 = qdiv(t, tn, itn, ti) << 4, n0 = ti << 4;
    const int m = m0 + li, n = n0 + li;
    const bool mv = m < Md, nv = n < Nd;
    // rows / columns past the matrix read row / column 0 instead: they only
    // feed outputs that are never stored
    const double* Ap = A + (mv ? m : 0) * sam + lk * sak;
    const double* Bp = B + (nv ? n : 0) * sbn + lk * sbk;
    const int da = 4 * sak, db = 4 * sbk, K4 = K & ~3;
    pg_d4 acc = {0.0, 0.0, 0.0, 0.0};
    int k0 = 0;
#pragma unroll 4
    for (; k0 < K4; k0 += 4) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(*Ap, *Bp, acc, 0, 0, 0);
      Ap += da;
      Bp += db;
    }
    if (k0 < K) {  // partial last step: k past K contributes zero
      double a = 0.0, b = 0.0;
      if (k0 + lk < K) {
        a = *Ap;
        b = *Bp;
      }
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (nv) {
      const int cno = mapoff(cn, n);
      // rows m0 + lk + 4 i, i < 4: one division for the four when they share
      // a block of the row map
      const int mr0 = m0 + lk;
      int r0;
      const int q0 = qdiv(mr0, cm.n0, cm.inv, r0);
      const int base = r0 * cm.s0 + q0 * cm.s1 + cno;
      const bool same = r0 + 12 < cm.n0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mr = mr0 + 4 * i;
        if (mr < Md) C[same ? base + 4 * i * cm.s0 : mapoff(cm, mr) + cno] = alpha * acc[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-core GEMM in reduced precision, float32 accumulation.
//   prec 1: float32 operands, v_mfma_f32_16x16x4f32 (lane l supplies
//           A[l%16][l/16], B[l/16][l%16])
//   prec 2: each float32 operand split into three bfloat16 pieces
//           x = hi + mid + lo (each rounded to nearest even from what the
//           previous pieces leave), which holds all 24 significand bits;
//           six bfloat16 products per tile, lo*hi + hi*lo + mid*mid +
//           mid*hi + hi*mid + hi*hi, smallest first (the dropped mid*lo,
//           lo*mid, lo*lo are below float32 rounding of the sum)
//   prec 3: single bfloat16 operands (8-bit significand)
//   prec 2 and 3 use v_mfma_f32_16x16x16bf16_1k (lane l supplies
//   A[l%16][4(l/16)+j], B[4(l/16)+j][l%16], j = 0..3).
// All hold D[4(l/16) + i][l%16] in accumulator element i.  Operands are
// float32 in memory; C has element type TC (float or double).
// ---------------------------------------------------------------------------
typedef float pg_f4 __attribute__((ext_vector_type(4)));
typedef short pg_s4 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (short)((u >> 16) | 0x40u);  // keep NaN a NaN
  const unsigned r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (short)(r >> 16);
}

__device__ inline float bf16_value(short h) {
  return __uint_as_float(((unsigned)(unsigned short)h) << 16);
}

template <int PREC, class TC>
__device__ inline void mgemm32(int Md, int Nd, int K, const float* A, int sam, int sak,
                               const float* B, int sbk, int sbn, TC* C, Map cm, Map cn,
                               float alpha, int tid, int nt, int rot = 0) {
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int tm = (Md + 15) >> 4, tn = (Nd + 15) >> 4;
  const float itn = 1.0f / (float)tn;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = (wave + nw - rot % nw) % nw; t < tm * tn; t += nw) {
    int ti;
    const int m0 = qdiv(t, tn, itn, ti) << 4, n0 = ti << 4;
    const int m = m0 + li, n = n0 + li;
    const bool mv = m < Md, nv = n < Nd;
    // rows / columns past the matrix read row / column 0 instead: they only
    // feed outputs that are never stored
    const float* Ap = A + (mv ? m : 0) * sam;
    const float* Bp = B + (nv ? n : 0) * sbn;
    pg_f4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == 1) {
      const float* Ak = Ap + lk * sak;
      const float* Bk = Bp + lk * sbk;
      const int da = 4 * sak, db = 4 * sbk, K4 = K & ~3;
      int k0 = 0;
#pragma unroll 4
      for (; k0 < K4; k0 += 4) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(*Ak, *Bk, acc, 0, 0, 0);
        Ak += da;
        Bk += db;
      }
      if (k0 < K) {  // partial last step: k past K contributes zero
        float a = 0.f, b = 0.f;
        if (k0 + lk < K) {
          a = *Ak;
          b = *Bk;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int k0 = 0; k0 < K; k0 += 16) {
        pg_s4 ah, bh, am, bm, al, bl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + 4 * lk + j;
          const float a = k < K ? Ap[k * sak] : 0.f;
          const float b = k < K ? Bp[k * sbk] : 0.f;
          ah[j] = bf16_rne(a);
          bh[j] = bf16_rne(b);
          if constexpr (PREC == 2) {
            const float ra = a - bf16_value(ah[j]), rb = b - bf16_value(bh[j]);
            am[j] = bf16_rne(ra);
            bm[j] = bf16_rne(rb);
            al[j] = bf16_rne(ra - bf16_value(am[j]));
            bl[j] = bf16_rne(rb - bf16_value(bm[j]));
          }
        }
        if constexpr (PREC == 2) {
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
      }
    }
    if (nv) {
      const int cno = mapoff(cn, n);
      // rows m0 + 4 lk + i, i < 4: one division for the four when they share
      // a block of the row map
      const int mr0 = m0 + 4 * lk;
      int r0;
      const int q0 = qdiv(mr0, cm.n0, cm.inv, r0);
      const int base = r0 * cm.s0 + q0 * cm.s1 + cno;
      const bool same = r0 + 3 < cm.n0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mr = mr0 + i;
        if (mr < Md) C[same ? base + i * cm.s0 : mapoff(cm, mr) + cno] = (TC)(alpha * acc[i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// reductions: lanes of a wave64 by butterfly shuffles, waves through LDS
// (red: at least nt/64 + 1 doubles); every thread receives the result.
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Make memory written by the lanes of this wave visible to the other lanes of
// the same wave (data passed through LDS between steps of a per-wave loop).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double block_sum(double v, double* red, int tid, int nt) {
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (nt + 63) >> 6; ++w) r += red[w];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* red, int tid, int nt) {
  v = wave_max(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (nt + 63) >> 6; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Householder LQ:  W (r x c, row-major, ld = c) = L (r x k) * Q (k x c),
// k = min(r, c), Q with orthonormal rows.  W is destroyed.  vbuf: k*c, tau: k,
// rowdot: r + k (>= max rows), red: nt.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lq_householder(double* W, int r, int c, double* Q, double* L, double* vbuf,
                                      double* tau, double* rowdot, double* red, int tid, int nt) {
  const int k = r < c ? r : c;
  for (int i = 0; i < k; ++i) {
    double part = 0.0;
    for (int t = i + 1 + tid; t < c; t += nt) part += W[i * c + t] * W[i * c + t];
    const double sigma = block_sum(part, red, tid, nt);
    const double alpha = W[i * c + i];
    double ti = 0.0, beta = alpha, scale = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      ti = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    for (int t = tid; t < c; t += nt)
      vbuf[i * c + t] = t < i ? 0.0 : (t == i ? 1.0 : W[i * c + t] * scale);
    __syncthreads();
    if (ti != 0.0) {
      // rows i+1..r-1:  w = W[row] . v ;  W[row] -= ti * w * v
      const int lane = tid & 63, nwv = (nt + 63) >> 6;
      for (int row = i + 1 + (tid >> 6); row < r; row += nwv) {
        double s = 0.0;
        for (int t = i + lane; t < c; t += 64) s += W[row * c + t] * vbuf[i * c + t];
        s = wave_sum(s);
        if (lane == 0) rowdot[row] = s;
      }
      __syncthreads();
      const int nrow = r - i - 1, ncol = c - i;
      for (int e = tid; e < nrow * ncol; e += nt) {
        const int row = i + 1 + e / ncol, t = i + e % ncol;
        W[row * c + t] -= ti * rowdot[row] * vbuf[i * c + t];
      }
    }
    __syncthreads();
    if (tid == 0) {
      W[i * c + i] = beta;
      tau[i] = ti;
    }
    for (int t = i + 1 + tid; t < c; t += nt) W[i * c + t] = 0.0;
    __syncthreads();
  }
  for (int e = tid; e < r * k; e += nt) {
    const int row = e / k, col = e % k;
    L[e] = col <= row ? W[row * c + col] : 0.0;
  }
  // Q = [I_k 0] H_{k-1} ... H_0
  for (int e = tid; e < k * c; e += nt) Q[e] = (e / c == e % c) ? 1.0 : 0.0;
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double ti = tau[i];
    if (ti == 0.0) continue;
    const int lane = tid & 63, nwv = (nt + 63) >> 6;
    for (int a = tid >> 6; a < k; a += nwv) {
      double s = 0.0;
      for (int t = i + lane; t < c; t += 64) s += Q[a * c + t] * vbuf[i * c + t];
      s = wave_sum(s);
      if (lane == 0) rowdot[a] = s;
    }
    __syncthreads();
    const int ncol = c - i;
    for (int e = tid; e < k * ncol; e += nt) {
      const int a = e / ncol, t = i + e % ncol;
      Q[a * c + t] -= ti * rowdot[a] * vbuf[i * c + t];
    }
    __syncthreads();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Leading eigenpairs of a symmetric matrix: Householder tridiagonalisation,
// bisection on Sturm counts, inverse iteration, back-transformation.
//
// G: n x n symmetric (ld = n), destroyed (its strictly lower part keeps the
// Householder vectors).  On exit lam[0..kk) holds the kk = min(n, k+1)
// largest eigenvalues in decreasing order and U orthonormal eigenvectors of
// the k largest, vector t at U[t*n .. t*n + n) (U: n k doubles).
// wk: sym_top_eig_work(n, k, nt) doubles; lw: max(3 n kb, 2 nt) doubles
// (U factors of kb inverse iterations at a time, kb >= 1; Sturm counts).
// ---------------------------------------------------------------------------
__host__ __device__ inline int sym_top_eig_work(int n, int k, int nt) {
  return 6 * n + 64 + 4 * (k + 2);
}

// Reciprocal by the hardware estimate refined with two Newton steps
// r <- r (2 - x r) (quadratic convergence; full double precision for the
// magnitudes met here, not correctly rounded).
__device__ inline double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}

// Inverse iteration for one eigenvalue of the tridiagonal (d, e): `iters`
// solves of (T - lam I) y = x from a fixed start vector, each by Gaussian
// elimination with partial pivoting fused with the forward substitution (a
// pivot below tiny is replaced by tiny), then back substitution with the
// stored reciprocal pivots.  Only the U factors are stored.  x: n, w: 3n.
// Sequential; recurrences in registers, row interchanges branch-free.
__device__ __forceinline__ void tri_inverse_iteration(const double* __restrict__ d,
                                                      const double* __restrict__ e, int n,
                                                      double lam, double tiny, int seed, int iters,
                                                      double* __restrict__ x,
                                                      double* __restrict__ w) {
  double* __restrict__ rdg = w;  // reciprocal pivots
  double* __restrict__ du = w + n;
  double* __restrict__ du2 = w + 2 * n;
  for (int i = 0; i < n; ++i) {
    const double h = (double)((i * 7919 + seed * 104729 + 17) % 1009) * (1.0 / 1009.0);
    x[i] = 1.0 + 0.5 * h;
  }
  for (int it = 0; it < iters; ++it) {
    double gi = d[0] - lam;          // current pivot candidate
    double ui = n > 1 ? e[0] : 0.0;  // its superdiagonal
    double xi = x[0];                // current right-hand side entry
#pragma unroll 4
    for (int i = 0; i + 1 < n; ++i) {
      const double li = e[i];
      const double gn = d[i + 1] - lam;
      const double un = i + 2 < n ? e[i + 1] : 0.0;
      const double xn = x[i + 1];
      // row interchange when the subdiagonal entry is the larger
      const bool sw = fabs(gi) < fabs(li);
      const double piv = sw ? li : gi, oth = sw ? gi : li;
      const double pg = fabs(piv) < tiny ? (piv < 0.0 ? -tiny : tiny) : piv;
      const double rp = recip_nr(pg);
      const double f = oth * rp;
      rdg[i] = rp;
      du[i] = sw ? gn : ui;
      du2[i] = sw ? un : 0.0;
      x[i] = sw ? xn : xi;
      const double xr = sw ? xi - f * xn : xn - f * xi;
      const double gr = sw ? ui - f * gn : gn - f * ui;
      ui = sw ? -f * un : un;
      xi = xr;
      gi = gr;
    }
    const double gl = fabs(gi) < tiny ? (gi < 0.0 ? -tiny : tiny) : gi;
    double a1 = xi * recip_nr(gl), a2 = 0.0;
    x[n - 1] = a1;
    double m = fabs(a1);
    if (n > 1) {
      const double v = (x[n - 2] - du[n - 2] * a1) * rdg[n - 2];
      x[n - 2] = v;
      a2 = a1;
      a1 = v;
      m = fmax(m, fabs(v));
    }
#pragma unroll 4
    for (int i = n - 3; i >= 0; --i) {
      const double v = (x[i] - du[i] * a1 - du2[i] * a2) * rdg[i];
      x[i] = v;
      a2 = a1;
      a1 = v;
      m = fmax(m, fabs(v));
    }
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (int i = 0; i < n; ++i) x[i] *= inv;
  }
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += x[i] * x[i];
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int i = 0; i < n; ++i) x[i] *= inv;
}

// Sturm counts: the number of eigenvalues of the tridiagonal (d, e2 = e^2)
// below each of four points x[0..3], as the number of sign changes of the
// leading principal minors p_i(x) = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}
// (p_{-1} = 0, p_0 = 1): no division.  The caller scales the matrix by a
// power of two to norm <= 1, so |p_i| grows at most threefold per step and a
// check every 8 steps, rescaling the pair (p_{i-1}, p_i) by an exact power of
// two when its larger member leaves [2^-500, 2^500], keeps it in range.  A
// minor that vanishes exactly counts as a sign change (the limit from below
// the eigenvalue of the leading block).  Four recurrences are interleaved.
__device__ inline void sturm_count4(const double* __restrict__ d, const double* __restrict__ e2,
                                    int n, const double* x, int* c) {
  double p0[4], p1[4];
  int cc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    p0[q] = 1.0;
    p1[q] = d[0] - x[q];
    if (p1[q] == 0.0) p1[q] = -0x1p-600;
    cc[q] = p1[q] < 0.0;
  }
  auto step = [&](double di, double ei) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double pn = (di - x[q]) * p1[q] - ei * p0[q];
      if (pn == 0.0) pn = p1[q] < 0.0 ? 0x1p-600 : -0x1p-600;
      cc[q] += (pn < 0.0) != (p1[q] < 0.0);
      p0[q] = p1[q];
      p1[q] = pn;
    }
  };
  int i = 1;
  // blocks of 8 steps: the block's d and e^2 are loaded together, then the range check
  for (; i + 8 <= n; i += 8) {
    double db[8], eb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      db[u] = d[i + u];
      eb[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) step(db[u], eb[u]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double a = fmax(fabs(p0[q]), fabs(p1[q]));
      if (a > 0x1p500 || a < 0x1p-500) {
        const int ex = ilogb(a);
        p0[q] = ldexp(p0[q], -ex);
        p1[q] = ldexp(p1[q], -ex);
      }
    }
  }
  for (; i < n; ++i) step(d[i], e2[i - 1]);
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = cc[q];
}

// Householder tridiagonalisation with the matrix held in registers: the 256
// threads form a 16 x 16 grid, thread (tr, tc) = (tid / 16, tid % 16) holding
// rows tr + 16 x and columns tc + 16 y (x, y < NB, n <= 16 NB), so the active
// part stays spread over all threads as it shrinks.  Per reflector: the
// column is published through LDS, one wave forms the reflector, then the
// product p = tau A v (row sums across the 16 lanes of a row group) and the
// rank-2 update A -= v w^T + w v^T run on the registers.  Output: d, e, tau,
// and reflector i (entries i+1 .. n-1, the first being 1) contiguous in row i
// of G (no longer needed once loaded).
template <int NB>
__device__ inline void tridiag_reg(double* G, int n, double* d, double* e, double* tau,
                                   double* vb, double* pv, double* colbuf, double* red, int tid) {
  const int tr = tid >> 4, tc = tid & 15, lane = tid & 63, wave = tid >> 6;
  double a[NB][NB];
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int r = tr + 16 * x, c = tc + 16 * y;
      a[x][y] = (r < n && c < n) ? G[r * n + c] : 0.0;
    }
  __syncthreads();
  for (int i = 0; i + 2 < n; ++i) {
    const int ib = i >> 4, ic = i & 15;
    // (1) column i, rows i .. n-1, to LDS
    if (tc == ic) {
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const int r = tr + 16 * x;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y) v = y == ib ? a[x][y] : v;
        if (r >= i && r < n) colbuf[r] = v;
      }
    }
    __syncthreads();
    // (2) reflector H = I - tau v v^T with v[i+1] = 1 mapping column i to beta e_{i+1}
    if (wave == 0) {
      double s = 0.0;
      for (int r = i + 2 + lane; r < n; r += 64) s += colbuf[r] * colbuf[r];
      s = wave_sum(s);
      const double alpha = colbuf[i + 1];
      double ti = 0.0, beta = alpha, scale = 0.0;
      if (s > 0.0) {
        const double nrm = sqrt(alpha * alpha + s);
        beta = alpha >= 0.0 ? -nrm : nrm;
        ti = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int r = lane; r < n; r += 64) {
        const double v = r <= i ? 0.0 : (r == i + 1 ? 1.0 : colbuf[r] * scale);
        vb[r] = v;
        if (r > i) G[i * n + (r - i - 1)] = v;  // reflector i, contiguous in row i of G
      }
      if (lane == 0) {
        tau[i] = ti;
        e[i] = beta;
        d[i] = colbuf[i];
      }
    }
    __syncthreads();
    const double ti = tau[i];
    if (ti == 0.0) continue;
    // (3) p = tau A v over the active block (v vanishes outside it)
    double vc[NB], ps[NB];
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int c = tc + 16 * y;
      vc[y] = c < n ? vb[c] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      double t = 0.0;
#pragma unroll
      for (int y = 0; y < NB; ++y) t += a[x][y] * vc[y];
      ps[x] = t;
    }
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      ps[x] += __shfl_xor(ps[x], 8, 64);
      ps[x] += __shfl_xor(ps[x], 4, 64);
      ps[x] += __shfl_xor(ps[x], 2, 64);
      ps[x] += __shfl_xor(ps[x], 1, 64);
    }
    double part = 0.0, vr[NB];
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      const int r = tr + 16 * x;
      vr[x] = r < n ? vb[r] : 0.0;
      ps[x] = (r > i && r < n) ? ti * ps[x] : 0.0;
      if (tc == 0) {
        if (r < n) pv[r] = ps[x];
        part += ps[x] * vr[x];
      }
    }
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    const double K = 0.5 * ti * (red[0] + red[1] + red[2] + red[3]);
    // (4) A -= v w^T + w v^T, w = p - K v
    double wc[NB];
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int c = tc + 16 * y;
      wc[y] = c < n ? pv[c] - K * vc[y] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      const double wr = ps[x] - K * vr[x];
#pragma unroll
      for (int y = 0; y < NB; ++y) a[x][y] -= vr[x] * wc[y] + wr * vc[y];
    }
  }
  // the last 2 x 2 block
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int r = tr + 16 * x, c = tc + 16 * y;
      if (r >= n - 2 && r < n && c == r) d[r] = a[x][y];
      if (r == n - 1 && c == n - 2) e[n - 2] = a[x][y];
    }
  if (tid == 0 && n >= 2) tau[n - 2] = 0.0;
  if (tid == 0 && n == 1) d[0] = a[0][0];
  __syncthreads();
}

__device__ __forceinline__ void sym_top_eig(double* G, int n, int k, double* lam, double* U, double* wk,
                                   double* lw, int kb, int tid, int nt) {
  const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
  double* d = wk;
  double* e = wk + n;
  double* e2 = wk + 2 * n;
  double* tau = wk + 3 * n;
  double* vb = wk + 4 * n;
  double* pv = wk + 5 * n;
  double* red = wk + 6 * n;             // nw partial sums (64 slots)
  double* iv = red + 64;                // 2 (k+2) interval ends
  double* cnt = lw;                     // Sturm counts (ints), then CGS coefficients
  double* Y = U;                        // eigenvectors of T, back-transformed in place
  const int kk = k + 1 < n ? k + 1 : n;

  // ---- 1. tridiagonalisation: G = Q T Q^T, Q = H_0 ... H_{n-3}
  // vrow: reflector i stored in row i of G (register path) rather than below
  // the subdiagonal of column i
  const bool vrow = nt == 256 && n <= 80;
  if (vrow) {
    // register-resident matrix (e2 serves as the column buffer until step 2)
    switch ((n + 15) >> 4) {
      case 1: tridiag_reg<1>(G, n, d, e, tau, vb, pv, e2, red, tid); break;
      case 2: tridiag_reg<2>(G, n, d, e, tau, vb, pv, e2, red, tid); break;
      case 3: tridiag_reg<3>(G, n, d, e, tau, vb, pv, e2, red, tid); break;
      case 4: tridiag_reg<4>(G, n, d, e, tau, vb, pv, e2, red, tid); break;
      default: tridiag_reg<5>(G, n, d, e, tau, vb, pv, e2, red, tid); break;
    }
  } else {
  for (int i = 0; i + 2 < n; ++i) {
    const int m = n - i - 1;
    if (wave == 0) {
      double s = 0.0;
      for (int r = 1 + lane; r < m; r += 64) {
        const double x = G[(i + 1 + r) * n + i];
        s += x * x;
      }
      s = wave_sum(s);
      const double alpha = G[(i + 1) * n + i];
      double ti = 0.0, beta = alpha, scale = 0.0;
      if (s > 0.0) {
        const double nrm = sqrt(alpha * alpha + s);
        beta = alpha >= 0.0 ? -nrm : nrm;
        ti = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int r = lane; r < m; r += 64) {
        const double v = r == 0 ? 1.0 : G[(i + 1 + r) * n + i] * scale;
        vb[r] = v;
        if (r > 0) G[(i + 1 + r) * n + i] = v;  // reflector kept below the subdiagonal
      }
      if (lane == 0) {
        tau[i] = ti;
        e[i] = beta;
      }
    }
    __syncthreads();
    const double ti = tau[i];
    if (ti != 0.0) {
      // p = ti * A22 v : groups of 8 lanes per row, plus per-wave partials of p.v
      double part = 0.0;
      for (int base = 0; base < m; base += nt / 8) {
        const int r = base + (tid >> 3);
        const int sub = tid & 7;
        double sacc = 0.0;
        if (r < m)
          for (int c = sub; c < m; c += 8) sacc += G[(i + 1 + r) * n + i + 1 + c] * vb[c];
        sacc += __shfl_xor(sacc, 1, 64);
        sacc += __shfl_xor(sacc, 2, 64);
        sacc += __shfl_xor(sacc, 4, 64);
        if (r < m && sub == 0) {
          pv[r] = ti * sacc;
          part += ti * sacc * vb[r];
        }
      }
      part = wave_sum(part);
      if (lane == 0) red[wave] = part;
      __syncthreads();
      double pdv = 0.0;
      for (int w = 0; w < nw; ++w) pdv += red[w];
      const double K = 0.5 * ti * pdv;
      // A22 -= v w^T + w v^T with w = p - K v
      // rows spread over waves, columns over lanes
      for (int r = wave; r < m; r += nw) {
        const double vr = vb[r], wr = pv[r] - K * vr;
        double* Gr = G + (i + 1 + r) * n + i + 1;
        for (int c = lane; c < m; c += 64) Gr[c] -= vr * (pv[c] - K * vb[c]) + wr * vb[c];
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += nt) {
    d[i] = G[i * n + i];
    if (i == n - 2) {
      e[i] = G[(n - 1) * n + n - 2];
      tau[i] = 0.0;
    }
  }
  __syncthreads();
  }
  for (int i = tid; i + 1 < n; i += nt) e2[i] = e[i] * e[i];
  __syncthreads();

  // ---- 2. the kk largest eigenvalues by multisection on Sturm counts
  double lo = 0.0, hi = 0.0, emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double off = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = i == 0 ? d[i] - off : fmin(lo, d[i] - off);
    hi = i == 0 ? d[i] + off : fmax(hi, d[i] + off);
    if (i + 1 < n) emax2 = fmax(emax2, e2[i]);
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 1e-290 * fmax(1.0, emax2);
  const double slack = 2.3e-16 * tnorm * n + 2.0 * pivmin;
  lo -= slack;
  hi += slack;
  // the matrix scaled by a power of two to norm <= 1 for the Sturm recurrences
  // (vb, pv are free after step 1)
  const double tsc = tnorm > 0.0 ? ldexp(1.0, -(ilogb(tnorm) + 1)) : 1.0;
  double* ds = vb;
  double* e2s = pv;
  for (int i = tid; i < n; i += nt) {
    ds[i] = d[i] * tsc;
    if (i + 1 < n) e2s[i] = e2[i] * (tsc * tsc);
  }
  if (tid < kk) {
    iv[2 * tid] = lo;
    iv[2 * tid + 1] = hi;
  }
  __syncthreads();
  // each thread evaluates 4 points; per target: 4 * (nt / kk) points per pass
  const int tpt = nt / kk < 63 ? nt / kk : 63;  // threads per target
  const int per = 4 * tpt;                       // evaluation points per target
  int* cnti = reinterpret_cast<int*>(cnt);       // nt * 4 ints fit in the nt + ... doubles region
  for (int it = 0; it < 40; ++it) {
    const int t = tid / tpt, g = tid - t * tpt;
    if (t < kk) {
      const double a = iv[2 * t], b = iv[2 * t + 1];
      double xs[4];
      for (int q = 0; q < 4; ++q) xs[q] = (a + (b - a) * (4 * g + q + 1) / (per + 1)) * tsc;
      int cc[4];
      sturm_count4(ds, e2s, n, xs, cc);
      for (int q = 0; q < 4; ++q) cnti[t * per + 4 * g + q] = cc[q];
    }
    __syncthreads();
    // new interval of target t: between the last point with count <= target and
    // the next one; the thread holding that point writes it
    double width = 0.0;
    if (t < kk) {
      const int target = n - 1 - t;
      const double a = iv[2 * t], b = iv[2 * t + 1];
      for (int q = 0; q < 4; ++q) {
        const int p = 4 * g + q;
        const bool le = cnti[t * per + p] <= target;
        const bool next_gt = p + 1 == per || cnti[t * per + p + 1] > target;
        const bool first_gt = p == 0 && !le;
        if ((le && next_gt) || first_gt) {
          const double lo2 = first_gt ? a : a + (b - a) * (p + 1) / (per + 1);
          const double hi2 = first_gt ? a + (b - a) / (per + 1)
                                      : (p + 1 == per ? b : a + (b - a) * (p + 2) / (per + 1));
          iv[2 * kk + 2 * t] = lo2;
          iv[2 * kk + 2 * t + 1] = hi2;
          width = (hi2 - lo2) > 1e-11 * fmax(fabs(lo2), fabs(hi2)) + 4.0 * pivmin ? 1.0 : 0.0;
        }
      }
    }
    __syncthreads();
    if (tid < kk) {
      iv[2 * tid] = iv[2 * kk + 2 * tid];
      iv[2 * tid + 1] = iv[2 * kk + 2 * tid + 1];
    }
    const double any = block_max(width, red, tid, nt);
    if (any == 0.0) break;
  }
  if (tid < kk) lam[tid] = 0.5 * (iv[2 * tid] + iv[2 * tid + 1]);
  __syncthreads();

  // ---- 3. eigenvectors of T: inverse iteration per eigenvalue, then CGS2
  const double tiny = fmax(2.3e-16 * tnorm, pivmin);
  for (int b0 = 0; b0 < k; b0 += kb) {
    const int t = b0 + tid;
    if (tid < kb && t < k) tri_inverse_iteration(d, e, n, lam[t], tiny, t, 2, Y + t * n, lw + tid * 3 * n);
    __syncthreads();
  }
  // Orthonormalisation.  Vectors of well separated eigenvalues are nearly
  // orthogonal already: two rounds of Cholesky QR (S = Y^T Y = L L^T on the
  // matrix cores, Y <- Y L^{-T}) finish them with a handful of barriers.  A
  // pivot of S below 1e-8 (vectors of a tight cluster, nearly parallel) sends
  // the whole set to classical Gram-Schmidt with reorthogonalisation instead.
  bool cholqr = 3 * n * kb >= k * k + 2 * k + 1;
  for (int round = 0; round < 2 && cholqr; ++round) {
    double* S = lw;           // k x k, lower triangle becomes L
    double* rdg = lw + k * k;  // 1 / L[t][t]
    double* okf = rdg + k;
    mgemm64(k, k, n, Y, n, 1, Y, 1, n, S, map1(k), map1(1), 1.0, tid, nt);
    __syncthreads();
    if (wave == 0) {
      bool ok = true;
      for (int c = 0; c < k; ++c) {
        const double s2 = S[c * k + c];
        ok = ok && s2 > 1e-8;
        const double piv = sqrt(fmax(s2, 1e-300));
        const double rp = 1.0 / piv;
        wave_sync();
        for (int r = c + 1 + lane; r < k; r += 64) S[r * k + c] *= rp;
        if (lane == 0) {
          S[c * k + c] = piv;
          rdg[c] = rp;
        }
        wave_sync();
        const int w = k - c - 1;
        for (int e2i = lane; e2i < w * w; e2i += 64) {
          const int r = c + 1 + e2i / w, q = c + 1 + e2i % w;
          if (q <= r) S[r * k + q] -= S[r * k + c] * S[q * k + c];
        }
        wave_sync();
      }
      if (lane == 0) okf[0] = ok ? 1.0 : 0.0;
    }
    __syncthreads();
    cholqr = okf[0] != 0.0;
    if (!cholqr) break;  // Y untouched by this round
    for (int r = tid; r < n; r += nt) {
      for (int t = 0; t < k; ++t) {
        double z = Y[t * n + r];
        for (int j = 0; j < t; ++j) z -= Y[j * n + r] * S[t * k + j];
        Y[t * n + r] = z * rdg[t];
      }
    }
    __syncthreads();
  }
  double* cf = lw + 3 * n;  // CGS coefficients (k), after the repair path's LU scratch
  for (int j = 0; j < k && !cholqr; ++j) {
    double* yj = Y + j * n;
    double nrm_before = 1.0;
    for (int pass = 0; pass < 2; ++pass) {
      // coefficients against the previous vectors, one wave per previous vector
      for (int i = wave; i < j; i += nw) {
        double s = 0.0;
        for (int r = lane; r < n; r += 64) s += Y[i * n + r] * yj[r];
        s = wave_sum(s);
        if (lane == 0) cf[i] = s;
      }
      __syncthreads();
      for (int r = tid; r < n; r += nt) {
        double v = yj[r];
        for (int i = 0; i < j; ++i) v -= cf[i] * Y[i * n + r];
        yj[r] = v;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int r = tid; r < n; r += nt) s += yj[r] * yj[r];
    s = block_sum(s, red, tid, nt);
    if (s < 1e-6 * nrm_before) {
      // a tight cluster: iterate again with the previous vectors projected out
      if (tid == 0) {
        double* w = lw;
        double t2 = 0.0;
        for (int rep = 0; rep < 3 && t2 <= 1e-6; ++rep) {
          tri_inverse_iteration(d, e, n, lam[j], tiny, j + 7 * (rep + 1), 2, yj, w);
          for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
              double c = 0.0;
              for (int r = 0; r < n; ++r) c += Y[i * n + r] * yj[r];
              for (int r = 0; r < n; ++r) yj[r] -= c * Y[i * n + r];
            }
          t2 = 0.0;
          for (int r = 0; r < n; ++r) t2 += yj[r] * yj[r];
        }
        // still inside the span (degenerate eigenvalue): the unit vector with the
        // largest remainder completes the orthonormal set
        for (int u = 0; u < n && t2 <= 1e-6; ++u) {
          for (int r = 0; r < n; ++r) yj[r] = r == u ? 1.0 : 0.0;
          for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
              double c = 0.0;
              for (int r = 0; r < n; ++r) c += Y[i * n + r] * yj[r];
              for (int r = 0; r < n; ++r) yj[r] -= c * Y[i * n + r];
            }
          t2 = 0.0;
          for (int r = 0; r < n; ++r) t2 += yj[r] * yj[r];
          if (t2 < 0.25) t2 = 0.0;
        }
      }
      __syncthreads();
      s = 0.0;
      for (int r = tid; r < n; r += nt) s += yj[r] * yj[r];
      s = block_sum(s, red, tid, nt);
    }
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int r = tid; r < n; r += nt) yj[r] *= inv;
    __syncthreads();
  }

  // ---- 4. back-transformation u = H_0 ... H_{n-3} y.
  // Register path (reflector i in row i of G): blocks of bb reflectors, last
  // block first, each applied as Q_blk = H_i0 ... H_{i0+bb-1} = I - V T V^T
  // (compact WY form, T upper triangular) through three small products on
  // the matrix cores.  Otherwise each wave carries up to four of its vectors
  // through every reflector.
  const int nref = n - 2;
  int bbk = 0;
  if (vrow && nref > 0) {
    for (int b = 16; b >= 8 && !bbk; b -= 8)
      if ((n - 1) * b + 2 * b * b + 2 * b * k <= 3 * n * kb) bbk = b;
  }
  if (bbk) {
    double* Vb = lw;                     // (n-1) x bbk, rows = absolute row i0+1+r
    double* VtV = Vb + (n - 1) * bbk;    // bbk x bbk
    double* Tm = VtV + bbk * bbk;        // bbk x bbk, upper
    double* W = Tm + bbk * bbk;          // bbk x k
    double* W2 = W + bbk * k;            // bbk x k
    for (int i1 = nref; i1 > 0; i1 -= bbk) {
      const int i0 = i1 > bbk ? i1 - bbk : 0, bb = i1 - i0, m = n - i0 - 1;
      // V: column j is reflector i0 + j, zero above its leading 1
      for (int q = tid; q < m * bb; q += nt) {
        const int r = q / bb, j = q - r * bb;  // absolute row R = i0 + 1 + r
        const int off = r - j;                 // R - (i0 + j) - 1
        Vb[r * bb + j] = off < 0 ? 0.0 : G[(i0 + j) * n + off];
      }
      __syncthreads();
      mgemm64(bb, bb, m, Vb, 1, bb, Vb, bb, 1, VtV, map1(bb), map1(1), 1.0, tid, nt);
      mgemm64(bb, k, m, Vb, 1, bb, Y + i0 + 1, 1, n, W, map1(k), map1(1), 1.0, tid, nt);
      __syncthreads();
      if (wave == 0) {
        for (int j = 0; j < bb; ++j) {
          const double tj = tau[i0 + j];
          double tij = 0.0;
          if (lane < j) {
            for (int l = lane; l < j; ++l) tij += Tm[lane * bb + l] * VtV[l * bb + j];
            tij *= -tj;
          }
          wave_sync();
          if (lane < bb) Tm[lane * bb + j] = lane < j ? tij : (lane == j ? tj : 0.0);
          wave_sync();
        }
      }
      __syncthreads();
      for (int q = tid; q < bb * k; q += nt) {
        const int j = q / k, t = q - j * k;
        double acc = 0.0;
        for (int l = j; l < bb; ++l) acc += Tm[j * bb + l] * W[l * k + t];
        W2[q] = acc;
      }
      __syncthreads();
      // Z = V W2 into the rows of G the remaining blocks no longer need
      double* Z = G + i0 * n;
      mgemm64(m, k, bb, Vb, bb, 1, W2, k, 1, Z, map1(k), map1(1), 1.0, tid, nt);
      __syncthreads();
      for (int q = tid; q < m * k; q += nt) {
        const int r = q / k, t = q - r * k;
        Y[t * n + i0 + 1 + r] -= Z[q];
      }
      __syncthreads();
    }
  }
  for (int t0 = wave; t0 < k && !bbk; t0 += 4 * nw) {
    const int t1 = t0 + nw, t2 = t0 + 2 * nw, t3 = t0 + 3 * nw;
    double* y0 = Y + t0 * n;
    double* y1 = Y + (t1 < k ? t1 : t0) * n;
    double* y2 = Y + (t2 < k ? t2 : t0) * n;
    double* y3 = Y + (t3 < k ? t3 : t0) * n;
    for (int i = n - 3; i >= 0; --i) {
      const double ti = tau[i];
      if (ti == 0.0) continue;
      const int m = n - i - 1;
      wave_sync();
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int r = lane; r < m; r += 64) {
        const double v = r == 0 ? 1.0 : G[vrow ? i * n + r : (i + 1 + r) * n + i];
        s0 += v * y0[i + 1 + r];
        s1 += v * y1[i + 1 + r];
        s2 += v * y2[i + 1 + r];
        s3 += v * y3[i + 1 + r];
      }
      s0 = wave_sum(s0) * ti;
      s1 = t1 < k ? wave_sum(s1) * ti : 0.0;
      s2 = t2 < k ? wave_sum(s2) * ti : 0.0;
      s3 = t3 < k ? wave_sum(s3) * ti : 0.0;
      wave_sync();
      for (int r = lane; r < m; r += 64) {
        const double v = r == 0 ? 1.0 : G[vrow ? i * n + r : (i + 1 + r) * n + i];
        y0[i + 1 + r] -= s0 * v;
        if (t1 < k) y1[i + 1 + r] -= s1 * v;
        if (t2 < k) y2[i + 1 + r] -= s2 * v;
        if (t3 < k) y3[i + 1 + r] -= s3 * v;
      }
    }
  }
  __syncthreads();
}

}  // namespace pg
