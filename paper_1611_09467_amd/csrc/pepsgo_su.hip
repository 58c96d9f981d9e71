// Simple-update imaginary-time evolution (the initialiser of Sec. III).
//
// The PEPS is held as site tensors Gamma [s][l][r][u][d] (the packed layout
// of the evaluation) and one weight vector lambda of length D per internal
// bond.  A step applies exp(-dtau J1 S.S) to every nearest-neighbour bond, in
// four groups of bonds that share no site (horizontal bonds with even column,
// odd column, then vertical bonds with even row, odd row), and cuts each bond
// back to D by an SVD.  The O(D^5) form of Sec. III: each site matrix
// M[(other legs), (s, bond leg)] (weights of the other legs absorbed) is
// reduced to its triangular factor R by Householder QR, the gate acts on the
// small R_A lambda R_B^T, whose SVD (one-sided Jacobi) gives the new weights
// and the new R factors, and the Householder reflectors carry those back to
// full site tensors; the other legs' weights are then divided out again
// (skipping weights <= 1e-12 of the bond's largest).  The new weights are the
// kept singular values over their 2-norm.
//
// One workgroup per bond; the site matrices live in a global workspace slot of
// the bond, the reduced matrices in LDS.
#include <math.h>

#include <algorithm>

#include "pepsgo_internal.h"
#include "pg_device.h"

namespace pg {

namespace {

constexpr int kSuThreads = 256;
constexpr int kSuMaxC = 2 * PEPSGO_MAX_D;  // columns (s, bond leg) of a site matrix
constexpr int kSuMaxN = 2 * kSuMaxC;       // side of the reduced two-site matrix
constexpr double kSuPinv = 1e-12;          // weights below this share of the largest are skipped
constexpr int kSuRed = kSuMaxC * 4 + kRedDoubles;
constexpr size_t kSuLdsBytes =
    sizeof(double) * (kSuRed + 3 * kSuMaxC + 2 * kSuMaxN * kSuMaxN + kSuMaxN + kSuMaxN / 2 + 8 +
                      2 * PEPSGO_MAX_D + 1);

struct SuArgs {
  int N, M, D;
  int kind;     // 0 horizontal, 1 vertical
  int parity;   // column (horizontal) or row (vertical) parity of the group
  double* G;    // packed Gamma
  const int64_t* site_off;
  double* lam;  // [nbonds][D]: horizontal bonds i*(M-1)+j, then vertical N*(M-1)+i*M+j
  double* ws;   // per bond: 4 site matrices of D^3 x 2D
  int64_t slot;
  double g[16];  // gate, row 2 s_a' + s_b', column 2 s_a + s_b
};

struct Site {
  int i, j;
  int dim[4];            // l, r, u, d
  const double* w[4];    // leg weights (nullptr on an open edge)
  int64_t off;
};

__device__ inline Site make_site(const SuArgs& a, int i, int j) {
  Site s;
  s.i = i;
  s.j = j;
  const int D = a.D, N = a.N, M = a.M;
  s.dim[0] = j == 0 ? 1 : D;
  s.dim[1] = j == M - 1 ? 1 : D;
  s.dim[2] = i == 0 ? 1 : D;
  s.dim[3] = i == N - 1 ? 1 : D;
  const int64_t hv = (int64_t)N * (M - 1);
  s.w[0] = j > 0 ? a.lam + ((int64_t)i * (M - 1) + j - 1) * D : nullptr;
  s.w[1] = j < M - 1 ? a.lam + ((int64_t)i * (M - 1) + j) * D : nullptr;
  s.w[2] = i > 0 ? a.lam + (hv + (int64_t)(i - 1) * M + j) * D : nullptr;
  s.w[3] = i < N - 1 ? a.lam + (hv + (int64_t)i * M + j) * D : nullptr;
  s.off = a.site_off[i * M + j];
  return s;
}

// largest weight of each leg, for the skip rule of the division
__device__ inline double wmax(const double* w, int n) {
  double m = 0.0;
  for (int k = 0; k < n; ++k) m = fmax(m, w[k]);
  return m;
}

// Site tensor element e -> (row of the other legs, s, bond-leg index) and the
// product of the other legs' weights (inverted with the skip rule when inv).
__device__ inline void site_index(const Site& S, int bl, int64_t e, int& row, int& s, int& x,
                                  double& w, bool inv, const double* wm) {
  int idx[4];
  int64_t r = e;
  for (int k = 3; k >= 0; --k) {
    idx[k] = (int)(r % S.dim[k]);
    r /= S.dim[k];
  }
  s = (int)r;
  x = idx[bl];
  row = 0;
  w = 1.0;
  for (int k = 0; k < 4; ++k) {
    if (k == bl) continue;
    row = row * S.dim[k] + idx[k];
    if (S.w[k]) {
      const double v = S.w[k][idx[k]];
      if (inv) w *= v > kSuPinv * wm[k] ? 1.0 / v : 0.0;
      else w *= v;
    }
  }
}

__device__ inline int64_t site_elems(const Site& S) {
  return 2LL * S.dim[0] * S.dim[1] * S.dim[2] * S.dim[3];
}

__device__ inline int other_rows(const Site& S, int bl) {
  int n = 1;
  for (int k = 0; k < 4; ++k)
    if (k != bl) n *= S.dim[k];
  return n;
}

// One Householder step on column k of X (rows x C, row-major): forms the
// reflector (stored below the diagonal, v_k = 1) and applies it to the
// columns right of k.  Returns tau.
__device__ double householder_step(double* X, int rows, int C, int k, double* red, int tid,
                                   int nt) {
  double part = 0.0;
  for (int i = k + 1 + tid; i < rows; i += nt) part += X[(int64_t)i * C + k] * X[(int64_t)i * C + k];
  const double tail = block_sum(part, red, tid, nt);
  const double alpha = X[(int64_t)k * C + k];
  if (tail == 0.0) return 0.0;  // column already reduced: H = I
  const double sigma = sqrt(alpha * alpha + tail);
  const double beta = alpha >= 0.0 ? -sigma : sigma;
  const double scale = 1.0 / (alpha - beta);
  const double tau = (beta - alpha) / beta;
  for (int i = k + 1 + tid; i < rows; i += nt) X[(int64_t)i * C + k] *= scale;
  __syncthreads();
  if (tid == 0) X[(int64_t)k * C + k] = beta;
  return tau;
}

// Y <- (I - tau v v^T) Y on columns [c0, C) of Y (rows x C), v from column k
// of V (v_k = 1, entries below k; V may be Y itself when c0 > k).  Row k of Y
// is copied first: every thread needs it while the thread owning it updates it.
__device__ void apply_reflector_safe(const double* V, int ldv, double* Y, int rows, int C, int c0,
                                     int k, double tau, double* red, double* rowk, int tid,
                                     int nt) {
  if (tau == 0.0 || c0 >= C) return;
  for (int c = tid; c < C; c += nt) rowk[c] = Y[(int64_t)k * C + c];
  __syncthreads();
  double p[kSuMaxC];
#pragma unroll
  for (int c = 0; c < kSuMaxC; ++c) p[c] = 0.0;
  for (int i = k + 1 + tid; i < rows; i += nt) {
    const double v = V[(int64_t)i * ldv + k];
#pragma unroll
    for (int c = 0; c < kSuMaxC; ++c)
      if (c >= c0 && c < C) p[c] += v * Y[(int64_t)i * C + c];
  }
  const int nw = (nt + 63) >> 6, wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < kSuMaxC; ++c) {
    if (c < c0 || c >= C) continue;
    const double v = wave_sum(p[c]);
    if ((tid & 63) == 0) red[c * nw + wave] = v;
  }
  __syncthreads();
  for (int i = k + tid; i < rows; i += nt) {
    const double v = i == k ? 1.0 : V[(int64_t)i * ldv + k];
    for (int c = c0; c < C; ++c) {
      double w = rowk[c];
      for (int q = 0; q < nw; ++q) w += red[c * nw + q];
      Y[(int64_t)i * C + c] -= tau * w * v;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kSuThreads) k_su_bond(SuArgs a) {
  extern __shared__ double lds[];
  double* red = lds;                           // kSuRed
  double* rowk = red + kSuRed;                 // kSuMaxC
  double* tauA = rowk + kSuMaxC;               // kSuMaxC
  double* tauB = tauA + kSuMaxC;               // kSuMaxC
  double* W = tauB + kSuMaxC;                  // reduced matrix, column-major, then rotated
  double* V = W + kSuMaxN * kSuMaxN;           // right rotations, column-major
  double* sig2 = V + kSuMaxN * kSuMaxN;        // kSuMaxN
  int* ord = reinterpret_cast<int*>(sig2 + kSuMaxN);  // kSuMaxN ints in kSuMaxN/2 doubles
  double* wmA = sig2 + kSuMaxN + kSuMaxN / 2;  // 4
  double* wmB = wmA + 4;                       // 4
  double* lamx = wmB + 4;                      // PEPSGO_MAX_D
  double* newlam = lamx + PEPSGO_MAX_D;        // PEPSGO_MAX_D
  int* rotated = reinterpret_cast<int*>(newlam + PEPSGO_MAX_D);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int D = a.D, C = 2 * D;

  // the bond of this workgroup
  int ia, ja, ib, jb, la, lb;
  int64_t bond;
  if (a.kind == 0) {
    const int per = (a.M - 1 - a.parity + 1) / 2;
    ia = blockIdx.x / per;
    ja = a.parity + 2 * (blockIdx.x % per);
    ib = ia;
    jb = ja + 1;
    la = 1;
    lb = 0;
    bond = (int64_t)ia * (a.M - 1) + ja;
  } else {
    ia = a.parity + 2 * (blockIdx.x / a.M);
    ja = blockIdx.x % a.M;
    ib = ia + 1;
    jb = ja;
    la = 3;
    lb = 2;
    bond = (int64_t)a.N * (a.M - 1) + (int64_t)ia * a.M + ja;
  }
  const Site SA = make_site(a, ia, ja), SB = make_site(a, ib, jb);
  const int nA = other_rows(SA, la), nB = other_rows(SB, lb);
  const int64_t R3 = (int64_t)D * D * D * C;
  double* MA = a.ws + (int64_t)blockIdx.x * 4 * R3;
  double* MB = MA + R3;
  double* YA = MB + R3;
  double* YB = YA + R3;
  double* lam = a.lam + bond * D;
  if (tid < 4) {
    wmA[tid] = SA.w[tid] ? wmax(SA.w[tid], SA.dim[tid]) : 1.0;
    wmB[tid] = SB.w[tid] ? wmax(SB.w[tid], SB.dim[tid]) : 1.0;
  }
  if (tid < D) lamx[tid] = lam[tid];

  // 1. site matrices with the other legs' weights absorbed
  {
    const int64_t eA = site_elems(SA), eB = site_elems(SB);
    for (int64_t e = tid; e < eA; e += nt) {
      int row, s, x;
      double w;
      site_index(SA, la, e, row, s, x, w, false, nullptr);
      MA[(int64_t)row * C + s * D + x] = a.G[SA.off + e] * w;
    }
    for (int64_t e = tid; e < eB; e += nt) {
      int row, s, x;
      double w;
      site_index(SB, lb, e, row, s, x, w, false, nullptr);
      MB[(int64_t)row * C + s * D + x] = a.G[SB.off + e] * w;
    }
  }
  __syncthreads();

  // 2. Householder QR of both (R in the upper triangle, reflectors below)
  const int KA = nA < C ? nA : C, KB = nB < C ? nB : C;
  for (int k = 0; k < KA; ++k) {
    const double t = householder_step(MA, nA, C, k, red, tid, nt);
    if (tid == 0) tauA[k] = t;
    __syncthreads();
    apply_reflector_safe(MA, C, MA, nA, C, k + 1, k, t, red, rowk, tid, nt);
  }
  for (int k = 0; k < KB; ++k) {
    const double t = householder_step(MB, nB, C, k, red, tid, nt);
    if (tid == 0) tauB[k] = t;
    __syncthreads();
    apply_reflector_safe(MB, C, MB, nB, C, k + 1, k, t, red, rowk, tid, nt);
  }

  // 3. reduced matrix W[(k, s_a'), (s_b', k')] = sum gate * R_A lambda R_B^T
  const int m = 2 * KA, n = 2 * KB;
  for (int e = tid; e < m * n; e += nt) {
    const int r = e % m, c = e / m;
    const int k = r >> 1, P = r & 1, Q = c / KB, kb = c % KB;
    double acc = 0.0;
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) {
        const double gv = a.g[(2 * P + Q) * 4 + 2 * p + q];
        if (gv == 0.0) continue;
        double t = 0.0;
        for (int x = 0; x < D; ++x) {
          const int ca = p * D + x, cb = q * D + x;
          const double ra = ca >= k ? MA[(int64_t)k * C + ca] : 0.0;
          const double rb = cb >= kb ? MB[(int64_t)kb * C + cb] : 0.0;
          t += ra * lamx[x] * rb;
        }
        acc += gv * t;
      }
    W[c * kSuMaxN + r] = acc;
  }
  for (int e = tid; e < n * n; e += nt) V[(e / n) * kSuMaxN + e % n] = (e / n) == (e % n) ? 1.0 : 0.0;
  __syncthreads();

  // 4. one-sided Jacobi on the columns of W (round-robin pairs, one pair per thread)
  const int nn = (n + 1) & ~1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) *rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < nn - 1; ++rnd) {
      if (tid < nn / 2) {
        int p, q;
        if (tid == 0) {
          p = nn - 1;
          q = rnd;
        } else {
          p = (rnd + tid) % (nn - 1);
          q = (rnd - tid + nn - 1) % (nn - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q < n) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int r = 0; r < m; ++r) {
            const double x = W[p * kSuMaxN + r], y = W[q * kSuMaxN + r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          if (ga != 0.0 && fabs(ga) > 1e-14 * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
            for (int r = 0; r < m; ++r) {
              const double x = W[p * kSuMaxN + r], y = W[q * kSuMaxN + r];
              W[p * kSuMaxN + r] = cs * x - sn * y;
              W[q * kSuMaxN + r] = sn * x + cs * y;
            }
            for (int r = 0; r < n; ++r) {
              const double x = V[p * kSuMaxN + r], y = V[q * kSuMaxN + r];
              V[p * kSuMaxN + r] = cs * x - sn * y;
              V[q * kSuMaxN + r] = sn * x + cs * y;
            }
            *rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    const int any = *rotated;
    __syncthreads();
    if (!any) break;
  }

  // 5. singular values, descending order, new weights
  for (int c = tid; c < n; c += nt) {
    double s = 0.0;
    for (int r = 0; r < m; ++r) s += W[c * kSuMaxN + r] * W[c * kSuMaxN + r];
    sig2[c] = s;
  }
  __syncthreads();
  const int keep = D < n ? (D < m ? D : m) : (n < m ? n : m);
  if (tid == 0) {
    for (int c = 0; c < n; ++c) ord[c] = c;
    for (int u = 0; u < keep; ++u) {
      int best = u;
      for (int c = u + 1; c < n; ++c)
        if (sig2[ord[c]] > sig2[ord[best]]) best = c;
      const int t = ord[u];
      ord[u] = ord[best];
      ord[best] = t;
    }
    double nrm = 0.0;
    for (int u = 0; u < keep; ++u) nrm += sig2[ord[u]];
    nrm = sqrt(nrm);
    for (int u = 0; u < D; ++u) newlam[u] = u < keep && nrm > 0.0 ? sqrt(sig2[ord[u]]) / nrm : 0.0;
  }
  __syncthreads();

  // 6. new R factors, padded with zero rows, carried back by the reflectors
  for (int64_t e = tid; e < (int64_t)nA * C; e += nt) {
    const int k = (int)(e / C), c = (int)(e % C), P = c / D, u = c % D;
    double v = 0.0;
    if (k < KA && u < keep) {
      const double s = sqrt(sig2[ord[u]]);
      if (s > 0.0) v = W[ord[u] * kSuMaxN + 2 * k + P] / s;
    }
    YA[e] = v;
  }
  for (int64_t e = tid; e < (int64_t)nB * C; e += nt) {
    const int k = (int)(e / C), c = (int)(e % C), Q = c / D, u = c % D;
    YB[e] = k < KB && u < keep && sig2[ord[u]] > 0.0 ? V[ord[u] * kSuMaxN + Q * KB + k] : 0.0;
  }
  __syncthreads();
  for (int k = KA - 1; k >= 0; --k)
    apply_reflector_safe(MA, C, YA, nA, C, 0, k, tauA[k], red, rowk, tid, nt);
  for (int k = KB - 1; k >= 0; --k)
    apply_reflector_safe(MB, C, YB, nB, C, 0, k, tauB[k], red, rowk, tid, nt);

  // 7. new weights, then the site tensors with the other legs' weights divided out
  if (tid < D) lam[tid] = newlam[tid];
  {
    const int64_t eA = site_elems(SA), eB = site_elems(SB);
    for (int64_t e = tid; e < eA; e += nt) {
      int row, s, x;
      double w;
      site_index(SA, la, e, row, s, x, w, true, wmA);
      a.G[SA.off + e] = YA[(int64_t)row * C + s * D + x] * w;
    }
    for (int64_t e = tid; e < eB; e += nt) {
      int row, s, x;
      double w;
      site_index(SB, lb, e, row, s, x, w, true, wmB);
      a.G[SB.off + e] = YB[(int64_t)row * C + s * D + x] * w;
    }
  }
}

// T = Gamma * prod over the legs of sqrt(lambda_leg), one thread per element
__global__ void __launch_bounds__(kSuThreads) k_su_absorb(SuArgs a, int64_t nparams, double* T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nparams) return;
  const int ns = a.N * a.M;
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.site_off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  const Site S = make_site(a, lo / a.M, lo % a.M);
  int64_t r = e - S.off;
  double w = 1.0;
  for (int k = 3; k >= 0; --k) {
    const int idx = (int)(r % S.dim[k]);
    r /= S.dim[k];
    if (S.w[k]) w *= sqrt(S.w[k][idx]);
  }
  T[e] = a.G[e] * w;
}

// The D-ramp: the same state at bond dimension Dt >= Df, inner legs padded with
// zeros; one thread per element of the larger tensors, then of the weights.
__global__ void __launch_bounds__(kSuThreads) k_su_pad(int N, int M, int Df, int Dt,
                                                       const int64_t* off_f, const int64_t* off_t,
                                                       int64_t nparams_t, const double* Gf,
                                                       double* Gt, const double* lamf,
                                                       double* lamt, int64_t nbonds) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nparams_t) {
    const int ns = N * M;
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off_t[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int i = lo / M, j = lo % M;
    const bool inner[4] = {j > 0, j < M - 1, i > 0, i < N - 1};
    int64_t r = e - off_t[lo];
    int idx[4];
    for (int k = 3; k >= 0; --k) {
      const int dt = inner[k] ? Dt : 1;
      idx[k] = (int)(r % dt);
      r /= dt;
    }
    bool in = true;
    int64_t src = r;  // the spin index
    for (int k = 0; k < 4; ++k) {
      const int df = inner[k] ? Df : 1;
      in = in && idx[k] < df;
      src = src * df + idx[k];
    }
    Gt[e] = in ? Gf[off_f[lo] + src] : 0.0;
  }
  if (e < nbonds * Dt) {
    const int64_t b = e / Dt;
    const int x = (int)(e % Dt);
    lamt[e] = x < Df ? lamf[b * Df + x] : 0.0;
  }
}

SuArgs su_args(int N, int M, int D, double* G, const int64_t* site_off, double* lam, double* ws,
               const double* gate) {
  SuArgs a;
  a.N = N;
  a.M = M;
  a.D = D;
  a.kind = 0;
  a.parity = 0;
  a.G = G;
  a.site_off = site_off;
  a.lam = lam;
  a.ws = ws;
  a.slot = 0;
  for (int k = 0; k < 16; ++k) a.g[k] = gate ? gate[k] : 0.0;
  return a;
}

}  // namespace

int64_t su_slots(int N, int M) {
  const int64_t h = (int64_t)N * (M / 2), v = (int64_t)((N) / 2) * M;
  return h > v ? h : v;
}

int64_t su_workspace_doubles(int N, int M, int D) {
  return su_slots(N, M) * 4 * (int64_t)D * D * D * 2 * D;
}

hipError_t launch_su_step(int N, int M, int D, double* G, const int64_t* site_off, double* lam,
                          double* ws, const double* gate, hipStream_t s) {
  SuArgs a = su_args(N, M, D, G, site_off, lam, ws, gate);
  for (int kind = 0; kind < 2; ++kind)
    for (int par = 0; par < 2; ++par) {
      int nb;
      if (kind == 0) nb = N * ((M - 1 - par + 1) / 2);
      else nb = ((N - 1 - par + 1) / 2) * M;
      if (nb <= 0) continue;
      a.kind = kind;
      a.parity = par;
      hipLaunchKernelGGL(k_su_bond, dim3(nb), dim3(kSuThreads), kSuLdsBytes, s, a);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t launch_su_absorb(int N, int M, int D, const double* G, const int64_t* site_off,
                            const double* lam, int64_t nparams, double* T, hipStream_t s) {
  SuArgs a = su_args(N, M, D, const_cast<double*>(G), site_off, const_cast<double*>(lam), nullptr,
                     nullptr);
  hipLaunchKernelGGL(k_su_absorb, dim3((unsigned)((nparams + kSuThreads - 1) / kSuThreads)),
                     dim3(kSuThreads), 0, s, a, nparams, T);
  return hipGetLastError();
}

hipError_t launch_su_pad(int N, int M, int Df, int Dt, const int64_t* off_f, const int64_t* off_t,
                         int64_t nparams_t, const double* Gf, double* Gt, const double* lamf,
                         double* lamt, hipStream_t s) {
  const int64_t nbonds = (int64_t)N * (M - 1) + (int64_t)(N - 1) * M;
  const int64_t n = std::max<int64_t>(nparams_t, nbonds * Dt);
  hipLaunchKernelGGL(k_su_pad, dim3((unsigned)((n + kSuThreads - 1) / kSuThreads)),
                     dim3(kSuThreads), 0, s, N, M, Df, Dt, off_f, off_t, nparams_t, Gf, Gt, lamf,
                     lamt, nbonds);
  return hipGetLastError();
}

}  // namespace pg
