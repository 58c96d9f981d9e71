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
struct Map {
  int n0, s0, s1;
};
__host__ __device__ inline Map map1(int s) { return Map{1 << 30, s, 0}; }
__host__ __device__ inline Map map2(int n0, int s0, int s1) { return Map{n0, s0, s1}; }
__device__ inline int mapoff(const Map& m, int i) {
  int q = i / m.n0;
  return (i - q * m.n0) * m.s0 + q * m.s1;
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
  for (int t = tid; t < tm * tn; t += nt) {
    const int mi = t / tn, ni = t - mi * tn;
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

// Tile shape picked from the problem shape (thin problems use thin tiles).
__device__ inline void gemm(const Gemm& g, int tid, int nt) {
  if (g.Md <= 0 || g.Nd <= 0) return;
  if (g.Nd <= 2)
    gemm_tiles<8, 1>(g, tid, nt);
  else if (g.Md <= 2)
    gemm_tiles<1, 8>(g, tid, nt);
  else
    gemm_tiles<4, 4>(g, tid, nt);
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
__device__ inline void lq_householder(double* W, int r, int c, double* Q, double* L, double* vbuf,
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
      for (int row = i + 1 + tid; row < r; row += nt) {
        double s = 0.0;
        for (int t = i; t < c; ++t) s += W[row * c + t] * vbuf[i * c + t];
        rowdot[row] = s;
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
    for (int a = tid; a < k; a += nt) {
      double s = 0.0;
      for (int t = i; t < c; ++t) s += Q[a * c + t] * vbuf[i * c + t];
      rowdot[a] = s;
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
// Cyclic parallel Jacobi eigensolver for a symmetric matrix.
// G: np x np (np even, ld = np), V: np x np.  On exit G is (numerically)
// diagonal with the eigenvalues and V holds the eigenvectors in its columns.
// Each round applies np/2 disjoint rotations (round-robin pairing), so every
// 2x2 block of G and every row pair of V is owned by one thread.
// cs: 2*(np/2) doubles, pq: np ints, flag: one int in LDS.
// A pair is rotated when |g_pq| > tol * sqrt(|g_pp g_qq|) and |g_pq| > floor_abs.
// ---------------------------------------------------------------------------
__device__ inline void jacobi_eig(double* G, double* V, int np, double* cs, int* pq, int* flag,
                                  double tol, double floor_abs, int max_sweeps, int tid,
                                  int nt) {
  const int h = np / 2;
  for (int e = tid; e < np * np; e += nt) V[e] = (e / np == e % np) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      for (int k = tid; k < h; k += nt) {
        int p, q;
        if (k == 0) {
          p = np - 1;
          q = round;
        } else {
          p = (round + k) % (np - 1);
          q = (round - k + (np - 1)) % (np - 1);
        }
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
        const double app = G[p * np + p], aqq = G[q * np + q], apq = G[p * np + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > floor_abs && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          *flag = 1;
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
      }
      __syncthreads();
      // G <- J^T G J on 2x2 blocks (a, b), a <= b; the block (b, a) is its transpose
      for (int blk = tid; blk < h * (h + 1) / 2; blk += nt) {
        // blk -> (a, b) with a <= b, row-major over the upper triangle
        int a = (int)((2 * h + 1 - sqrt((double)((2 * h + 1) * (2 * h + 1) - 8 * blk))) / 2);
        while (a > 0 && a * h - a * (a - 1) / 2 > blk) --a;
        while ((a + 1) * h - (a + 1) * a / 2 <= blk) ++a;
        const int b = a + blk - (a * h - a * (a - 1) / 2);
        const double ca = cs[2 * a], sa = cs[2 * a + 1], cb = cs[2 * b], sb = cs[2 * b + 1];
        if (sa == 0.0 && sb == 0.0) continue;
        const int pa = pq[2 * a], qa = pq[2 * a + 1], pb = pq[2 * b], qb = pq[2 * b + 1];
        const double b00 = G[pa * np + pb], b01 = G[pa * np + qb];
        const double b10 = G[qa * np + pb], b11 = G[qa * np + qb];
        // T = B * Rb, Rb = [[cb, sb], [-sb, cb]]
        const double t00 = cb * b00 - sb * b01, t01 = sb * b00 + cb * b01;
        const double t10 = cb * b10 - sb * b11, t11 = sb * b10 + cb * b11;
        // B' = Ra^T T
        const double n00 = ca * t00 - sa * t10, n11 = sa * t01 + ca * t11;
        double n01 = ca * t01 - sa * t11, n10 = sa * t00 + ca * t10;
        if (a == b) {
          if (sa != 0.0) {
            n01 = 0.0;
            n10 = 0.0;
          }
          G[pa * np + pa] = n00;
          G[pa * np + qa] = n01;
          G[qa * np + pa] = n10;
          G[qa * np + qa] = n11;
        } else {
          G[pa * np + pb] = n00;
          G[pa * np + qb] = n01;
          G[qa * np + pb] = n10;
          G[qa * np + qb] = n11;
          G[pb * np + pa] = n00;
          G[qb * np + pa] = n01;
          G[pb * np + qa] = n10;
          G[qb * np + qa] = n11;
        }
      }
      // V <- V J
      for (int e = tid; e < np * h; e += nt) {
        const int row = e / h, a = e - row * h;
        const double ca = cs[2 * a], sa = cs[2 * a + 1];
        if (sa == 0.0) continue;
        const int pa = pq[2 * a], qa = pq[2 * a + 1];
        const double vp = V[row * np + pa], vq = V[row * np + qa];
        V[row * np + pa] = ca * vp - sa * vq;
        V[row * np + qa] = sa * vp + ca * vq;
      }
      __syncthreads();
    }
    const int any = *flag;
    __syncthreads();
    if (!any) break;
  }
}

// order[0..n) = indices of the diagonal of G (ld = np) by decreasing value
// (ties by index).  order: n ints.
__device__ inline void sort_desc(const double* G, int np, int n, int* order, int tid, int nt) {
  for (int i = tid; i < n; i += nt) {
    const double vi = G[i * np + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double vj = G[j * np + j];
      rank += (vj > vi) || (vj == vi && j < i);
    }
    order[rank] = i;
  }
  __syncthreads();
}

}  // namespace pg
