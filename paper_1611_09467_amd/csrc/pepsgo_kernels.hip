// Per-sample kernels of the boundary-MPS evaluation (one workgroup per sample).
//
//   k_edges     U_0 and Dn_{N-1}: the first and last rows read as MPSs
//   k_zip       absorb a row into a boundary MPS: exact LQ sweep to
//               right-canonical form, then zip-up with SVD truncation to Dc
//               (Fig. 1(d) of the paper; truncated SVD of each block X by
//               Householder bidiagonalisation, bisection on Sturm counts and
//               inverse iteration on the Golub-Kahan tridiagonal)
//   k_sandwich  <U_{i-1}| row i |Dn_{i+1}>: psi_i, Delta_ij = B_ij / psi_i
//               (Eqs. (4)-(5)), horizontal exchange ratios
//   k_strip     <U_{i-1}| rows i, i+1 |Dn_{i+2}>: vertical and diagonal
//               exchange ratios
//   k_finalize  E(S) assembly for Eq. (7), outputs and flags
#include <math.h>

#include <map>
#include <mutex>

#include "pepsgo_internal.h"
#include "pg_device.h"

namespace pg {

// 3- and 4-leg tensor views (pointer, dimensions, strides)
struct T3 {
  const double* p;
  int d0, d1, d2, s0, s1, s2;
};
struct T4 {
  const double* p;
  int d0, d1, d2, d3, s0, s1, s2, s3;
};

__device__ inline double* sample_ws(const Lat& L) { return L.ws + (int64_t)blockIdx.x * L.ws_stride; }
__device__ inline double* env_site(const Lat& L, double* ws, int slot, int j) {
  return ws + L.off_env + (int64_t)slot * L.env_stride + (int64_t)j * L.site_slot;
}
__device__ inline uint8_t spin(const Lat& L, int i, int j) {
  return L.cfg[(int64_t)blockIdx.x * L.N * L.M + i * L.M + j];
}
// slice T_ij[s] as a [l][r][u][d] view
__device__ inline T4 slice(const Lat& L, int i, int j, int s) {
  int dl, dr, du, dd;
  site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
  const double* p = L.T + L.site_off[i * L.M + j] + (int64_t)s * dl * dr * du * dd;
  return T4{p, dl, dr, du, dd, dr * du * dd, du * dd, dd, 1};
}
// the same slice with left/right legs exchanged (used by right-to-left sweeps)
__device__ inline T4 mirror(const T4& a) {
  return T4{a.p, a.d1, a.d0, a.d2, a.d3, a.s1, a.s0, a.s2, a.s3};
}
// MPS site tensor [a][p][b] as a left view (a, p, b) or right view (b, p, a)
__device__ inline T3 mps_left(const double* p, int a, int ph, int b) {
  return T3{p, a, ph, b, ph * b, b, 1};
}
__device__ inline T3 mps_right(const double* p, int a, int ph, int b) {
  return T3{p, b, ph, a, 1, b, ph * b};
}

__device__ inline double* bufp(const BufPlan& bp, double* lds, double* gscr, int i) {
  return ((bp.glob >> i) & 1u) ? gscr + bp.off[i] : lds + bp.off[i];
}

// The same with the placement known at compile time (GM = the plan's glob
// mask): LDS-resident buffers are then plain LDS pointers and their accesses
// compile to LDS instructions; kGlobAny keeps the run-time choice.
constexpr uint32_t kGlobAny = 0xFFFFFFFFu;
template <uint32_t GM>
__device__ inline double* bufp_t(const BufPlan& bp, double* lds, double* gscr, int i) {
  if constexpr (GM == kGlobAny)
    return bufp(bp, lds, gscr, i);
  else
    return ((GM >> i) & 1u) ? gscr + bp.off[i] : lds + bp.off[i];
}

// Copy a tensor view into contiguous LDS (logical leg order) and return a view
// of the copy; the caller synchronises before reading it.
__device__ inline T3 stage3(const T3& v, double* dst, int tid, int nt) {
  const int n12 = v.d1 * v.d2, n = v.d0 * n12;
  const float i12 = 1.0f / (float)n12, i2f = 1.0f / (float)v.d2;
  for (int e = tid; e < n; e += nt) {
    int rem, i2;
    const int i0 = qdiv(e, n12, i12, rem), i1 = qdiv(rem, v.d2, i2f, i2);
    dst[e] = v.p[i0 * v.s0 + i1 * v.s1 + i2 * v.s2];
  }
  return T3{dst, v.d0, v.d1, v.d2, n12, v.d2, 1};
}
__device__ inline T4 stage4(const T4& v, double* dst, int tid, int nt) {
  const int n23 = v.d2 * v.d3, n123 = v.d1 * n23, n = v.d0 * n123;
  const float i123 = 1.0f / (float)n123, i23 = 1.0f / (float)n23, i3f = 1.0f / (float)v.d3;
  for (int e = tid; e < n; e += nt) {
    int r1, r2, i3;
    const int i0 = qdiv(e, n123, i123, r1), i1 = qdiv(r1, n23, i23, r2);
    const int i2 = qdiv(r2, v.d3, i3f, i3);
    dst[e] = v.p[i0 * v.s0 + i1 * v.s1 + i2 * v.s2 + i3 * v.s3];
  }
  return T4{dst, v.d0, v.d1, v.d2, v.d3, n123, n23, v.d3, 1};
}

// ---------------------------------------------------------------------------
// one column of a row sandwich:  Eout[x][r][y] = sum Ein[a][l][b] U[a][u][x] A[l][r][u][d] Dn[b][d][y]
// on the float64 matrix cores.  Every intermediate is written in the layout
// that makes the next product's operands single-stride:
//   T1[(l u)][(b x)] = sum_a      Ein[a][(l b)] U[a][(u x)]
//   T2[(x r)][(b d)] = sum_(l u)  T1[(l u)][(b x)] A[(l u)][(r d)]     (A staged [l][u][r][d])
//   Eout[(x r)][y]   = sum_(b d)  T2[(x r)][(b d)] Dn[(b d)][y]
// ---------------------------------------------------------------------------
__device__ inline void upd1_t1(const double* Ein, const T3& U0, int Ld, int Bd, double* T1,
                               double* stg, int tid, int nt) {
  const T3 U = stage3(U0, stg, tid, nt);
  __syncthreads();
  const int Ad = U.d0, Ud = U.d1, Xd = U.d2;
  mgemm64(Ld * Bd, Ud * Xd, Ad, Ein, 1, Ld * Bd, U.p, Ud * Xd, 1, T1, map2(Bd, Xd, Ud * Bd * Xd),
          map2(Xd, 1, Bd * Xd), 1.0, tid, nt);
  __syncthreads();
}

__device__ inline void upd1_rest(const double* T1, int Ud, int Xd, const T4& A0, const T3& Dn0,
                                 double* T2, double* Eout, double* stg, int tid, int nt) {
  // A staged with its legs in the order [l][u][r][d]
  const T4 Au{A0.p, A0.d0, A0.d2, A0.d1, A0.d3, A0.s0, A0.s2, A0.s1, A0.s3};
  const T4 A = stage4(Au, stg, tid, nt);
  const T3 Dn = stage3(Dn0, stg + A0.d0 * A0.d1 * A0.d2 * A0.d3, tid, nt);
  __syncthreads();
  const int Ld = A0.d0, Rd = A0.d1, Dd = A0.d3, Bd = Dn.d0, Yd = Dn.d2;
  mgemm64(Bd * Xd, Rd * Dd, Ld * Ud, T1, 1, Bd * Xd, A.p, Rd * Dd, 1, T2,
          map2(Xd, Rd * Bd * Dd, Dd), map2(Dd, 1, Bd * Dd), 1.0, tid, nt);
  __syncthreads();
  mgemm64(Xd * Rd, Yd, Bd * Dd, T2, Bd * Dd, 1, Dn.p, Yd, 1, Eout, map1(Yd), map1(1), 1.0, tid,
          nt);
  __syncthreads();
}

__device__ inline void update1(const double* Ein, const T3& U, const T4& A, const T3& Dn,
                               double* T1, double* T2, double* Eout, double* stg, int tid, int nt) {
  upd1_t1(Ein, U, A.d0, Dn.d0, T1, stg, tid, nt);
  upd1_rest(T1, U.d1, U.d2, A, Dn, T2, Eout, stg, tid, nt);
}

// ---------------------------------------------------------------------------
// one column of a two-row strip:
// Eout[x][r1][r2][y] = sum Ein[a][l1][l2][b] U[a][u][x] A1[l1][r1][u][m] A2[l2][r2][m][d] Dn[b][d][y]
// computed one x at a time on the matrix cores.  The operands are staged in
// LDS and every intermediate is written in the layout that makes the next
// contraction index contiguous:
//   S1  T1[(l2 b)][(l1 u)] = sum_a   Ein[a][(l1 l2 b)] U[a][u][x]
//   S2  T2[(b r1)][(l2 m)] = sum_(l1 u) T1[(l2 b)][(l1 u)] A1[(l1 u)][(r1 m)]
//   S3  T3[(r1 r2)][(b d)] = sum_(l2 m) T2[(b r1)][(l2 m)] A2[(l2 m)][(r2 d)]
//   S4  Eout[x][(r1 r2)][y] = sum_(b d) T3[(r1 r2)][(b d)] Dn[(b d)][y]
// Leading dimensions are odd so that rows fall in distinct LDS banks.
// ---------------------------------------------------------------------------
__device__ inline int odd_ld(int n) { return n | 1; }
__device__ inline int tiles16(int m, int n) { return ((m + 15) >> 4) * ((n + 15) >> 4); }

// element type of the strip contractions: float64 (0); float32 storage for
// the float32 (1), split-bfloat16 (2) and bfloat16 (3) matrix-core products
template <int PREC> struct PT { typedef float T; };
template <> struct PT<0> { typedef double T; };

template <int PREC, class TC>
__device__ inline void pgemm(int Md, int Nd, int K, const typename PT<PREC>::T* A, int sam, int sak,
                             const typename PT<PREC>::T* B, int sbk, int sbn, TC* C, Map cm,
                             Map cn, double alpha, int tid, int nt, int rot = 0) {
  if constexpr (PREC == 0)
    mgemm64(Md, Nd, K, A, sam, sak, B, sbk, sbn, C, cm, cn, alpha, tid, nt, rot);
  else
    mgemm32<PREC, TC>(Md, Nd, K, A, sam, sak, B, sbk, sbn, C, cm, cn, (float)alpha, tid, nt, rot);
}

template <int PREC>
__device__ inline void update2(const typename PT<PREC>::T* Ein, const T3& U, const T4& A1,
                               const T4& A2, const T3& Dn, typename PT<PREC>::T* T1,
                               typename PT<PREC>::T* T2, typename PT<PREC>::T* Eout,
                               typename PT<PREC>::T* stg, int xc, int tid, int nt) {
  typedef typename PT<PREC>::T T;
  const int Ad = U.d0, Ud = U.d1, Xd = U.d2;
  const int L1 = A1.d0, R1 = A1.d1, Mm = A1.d3;
  const int L2 = A2.d0, R2 = A2.d1, Dd = A2.d3;
  const int Bd = Dn.d0, Yd = Dn.d2;
  // staging: sU[a][(x u)], sA1[(l1 u)][(r1 m)], sA2[(l2 m)][(r2 d)], sDn[(b d)][y]
  T* sU = stg;
  T* sA1 = sU + Xd * Ad * Ud;
  T* sA2 = sA1 + L1 * Ud * R1 * Mm;
  T* sDn = sA2 + L2 * Mm * R2 * Dd;
  // index decompositions by float reciprocals (qdiv)
  const float iXU = 1.0f / (float)(Xd * Ud), iU = 1.0f / (float)Ud, iRM = 1.0f / (float)(R1 * Mm);
  const float iM = 1.0f / (float)Mm, iRD = 1.0f / (float)(R2 * Dd), iD = 1.0f / (float)Dd;
  const float iY = 1.0f / (float)Yd;
  for (int e = tid; e < Xd * Ad * Ud; e += nt) {
    int r, u;
    const int a = qdiv(e, Xd * Ud, iXU, r), x = qdiv(r, Ud, iU, u);
    sU[e] = (T)U.p[a * U.s0 + u * U.s1 + x * U.s2];
  }
  for (int e = tid; e < L1 * Ud * R1 * Mm; e += nt) {
    int n, u, m;
    const int k = qdiv(e, R1 * Mm, iRM, n);
    const int l = qdiv(k, Ud, iU, u), r = qdiv(n, Mm, iM, m);
    sA1[e] = (T)A1.p[l * A1.s0 + r * A1.s1 + u * A1.s2 + m * A1.s3];
  }
  for (int e = tid; e < L2 * Mm * R2 * Dd; e += nt) {
    int n, m, d;
    const int k = qdiv(e, R2 * Dd, iRD, n);
    const int l = qdiv(k, Mm, iM, m), r = qdiv(n, Dd, iD, d);
    sA2[e] = (T)A2.p[l * A2.s0 + r * A2.s1 + m * A2.s2 + d * A2.s3];
  }
  for (int e = tid; e < Bd * Dd * Yd; e += nt) {
    int y, d;
    const int k = qdiv(e, Yd, iY, y), b = qdiv(k, Dd, iD, d);
    sDn[e] = (T)Dn.p[b * Dn.s0 + d * Dn.s1 + y * Dn.s2];
  }
  __syncthreads();
  const int ld1 = odd_ld(L1 * Ud), ld2 = odd_ld(L2 * Mm), ld3 = odd_ld(Bd * Dd);
  // per-x slots of the intermediates: xc values of x run through each stage
  // between two barriers (their products are independent)
  const int s1 = L2 * Bd * ld1 > R1 * R2 * ld3 ? L2 * Bd * ld1 : R1 * R2 * ld3;
  const int s2 = Bd * R1 * ld2;
  for (int x0 = 0; x0 < Xd; x0 += xc) {
    const int nx = Xd - x0 < xc ? Xd - x0 : xc;
    // S1 for the whole chunk: columns (x u), x-slot q of T1 at T1 + q s1
    pgemm<PREC, T>(L1 * L2 * Bd, nx * Ud, Ad, Ein, 1, L1 * L2 * Bd, sU + x0 * Ud, Xd * Ud, 1, T1,
                   map2(L2 * Bd, ld1, Ud), map2(Ud, 1, s1), 1.0, tid, nt);
    __syncthreads();
    for (int q = 0; q < nx; ++q)
      pgemm<PREC, T>(L2 * Bd, R1 * Mm, L1 * Ud, T1 + q * s1, ld1, 1, sA1, R1 * Mm, 1, T2 + q * s2,
                     map2(Bd, R1 * ld2, Mm), map2(Mm, 1, ld2), 1.0, tid, nt,
                     q * tiles16(L2 * Bd, R1 * Mm));
    __syncthreads();
    // the third product overwrites the first one's slot (dead by now)
    for (int q = 0; q < nx; ++q)
      pgemm<PREC, T>(Bd * R1, R2 * Dd, L2 * Mm, T2 + q * s2, ld2, 1, sA2, R2 * Dd, 1, T1 + q * s1,
                     map2(R1, R2 * ld3, Dd), map2(Dd, 1, ld3), 1.0, tid, nt,
                     q * tiles16(Bd * R1, R2 * Dd));
    __syncthreads();
    for (int q = 0; q < nx; ++q)
      pgemm<PREC, T>(R1 * R2, Yd, Bd * Dd, T1 + q * s1, ld3, 1, sDn, Yd, 1,
                     Eout + (int64_t)(x0 + q) * R1 * R2 * Yd, map1(Yd), map1(1), 1.0, tid, nt,
                     q * tiles16(R1 * R2, Yd));
    __syncthreads();
  }
}

// scale v[0..n) by 1/max|v|; returns ln(max|v|) (or -inf / nan for 0 / non-finite)
template <class T>
__device__ inline double normalise(T* v, int n, double* red, int tid, int nt) {
  double m = 0.0;
  for (int e = tid; e < n; e += nt) {
    const double a = fabs((double)v[e]);
    m = (a > m || a != a) ? a : m;
  }
  m = block_max(m, red, tid, nt);
  if (!(m > 0.0) || !isfinite(m)) return m == 0.0 ? -INFINITY : NAN;
  const T inv = (T)(1.0 / m);
  for (int e = tid; e < n; e += nt) v[e] *= inv;
  __syncthreads();
  return log(m);
}

template <class T>
__device__ inline double dot(const T* a, const T* b, int n, double* red, int tid, int nt) {
  double s = 0.0;
  for (int e = tid; e < n; e += nt) s += (double)a[e] * (double)b[e];
  return block_sum(s, red, tid, nt);
}

// Kernels of one sample may run on concurrent streams: flags are set atomically.
__device__ inline void set_flag(double* ws, const Lat& L, uint32_t f, int tid) {
  if (tid == 0) atomicOr(reinterpret_cast<uint32_t*>(ws + L.off_flags), f);
}
__device__ inline bool sample_dead(double* ws, const Lat& L) {
  const uint32_t f = *reinterpret_cast<const uint32_t*>(ws + L.off_flags);
  return (f & (kFlagZero | kFlagNonfinite)) != 0;
}

// ---------------------------------------------------------------------------
// k_edges
// ---------------------------------------------------------------------------
// U_0 into slot_top0 and Dn_{N-1} into slot_bot (a negative slot is not
// written); reset: start a sample (flags, markers, energy, log-scales cleared)
__global__ void __launch_bounds__(kThreads) k_edges(Lat L, int slot_top0, int slot_bot, int reset) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  if (tid == 0 && reset) {
    *reinterpret_cast<uint32_t*>(ws + L.off_flags) = 0u;
    ws[L.off_flags + 1] = 0.0;
    ws[L.off_flags + 2] = NAN;
    ws[L.off_eloc] = 0.0;
    if (slot_top0 >= 0) ws[L.off_envlog + slot_top0] = 0.0;
    if (slot_bot >= 0) ws[L.off_envlog + slot_bot] = 0.0;
  }
  for (int j = 0; j < L.M; ++j) {
    if (slot_top0 >= 0) {
      // U_0 site j: [l][d][r] from A_0j[l][r][u=0][d]
      const T4 a = slice(L, 0, j, spin(L, 0, j));
      double* o = env_site(L, ws, slot_top0, j);
      for (int e = tid; e < a.d0 * a.d3 * a.d1; e += nt) {
        const int l = e / (a.d3 * a.d1), rem = e - l * a.d3 * a.d1, d = rem / a.d1, r = rem - d * a.d1;
        o[e] = a.p[l * a.s0 + r * a.s1 + d * a.s3];
      }
    }
    if (slot_bot >= 0) {
      // Dn_{N-1} site j: [l][u][r] from A_{N-1,j}[l][r][u][d=0]
      const T4 c = slice(L, L.N - 1, j, spin(L, L.N - 1, j));
      double* q = env_site(L, ws, slot_bot, j);
      for (int e = tid; e < c.d0 * c.d2 * c.d1; e += nt) {
        const int l = e / (c.d2 * c.d1), rem = e - l * c.d2 * c.d1, u = rem / c.d1, r = rem - u * c.d1;
        q[e] = c.p[l * c.s0 + r * c.s1 + u * c.s2];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_zip
// ---------------------------------------------------------------------------
// NT = 256: one workgroup of four waves per sample.  NT = 64: one wave per
// sample (blocks up to 72 x 72 held in the wave's registers during the
// bidiagonalisation), eight samples per CU.
template <uint32_t GM, int NT>
__global__ void __launch_bounds__(NT, 2) k_zip(Lat L, ZipShape z, BufPlan bp) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  constexpr int nt = NT;
  double* ws = sample_ws(L);
  if (sample_dead(ws, L)) return;
  double* gscr = ws + L.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, ZB_RED);
  double* bG = bufp_t<GM>(bp, lds, gscr, ZB_G);
  double* bV = bufp_t<GM>(bp, lds, gscr, ZB_V);
  double* bX = bufp_t<GM>(bp, lds, gscr, ZB_X);
  double* bC = bufp_t<GM>(bp, lds, gscr, ZB_C);
  // eigenvectors (vector t at bUk + t * rows) follow the eigensolver work area
  double* bUk = bV + top_svd_work(L.chimax * L.D, L.chimax * L.D, L.chimax, NT == 64);
  double* misc = bufp_t<GM>(bp, lds, gscr, ZB_MISC);
  double* bLW = bufp_t<GM>(bp, lds, gscr, ZB_LW);
  const int M = L.M, k = z.row, chm = L.chimax;
  double* lam = misc;                                    // chimax + 1
  double* tau = misc + chm + 2;                          // chimax
  double* rowdot = tau + chm;                            // 2 * chimax

  // ---- phase A: exact LQ sweep of the input MPS into the temporary slot
  double* Lc = bC;
  double* Ln = bC + chm * chm;
  for (int j = M - 1; j >= 0; --j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, k, j, &dl, &dr, &du, &dd);
    const int p = z.dir == 0 ? du : dd;
    const int r = z.chi_in[j], cR = z.chic[j + 1], cRin = z.chi_in[j + 1];
    const double* Min = env_site(L, ws, z.in_slot, j);
    double* W = bG;
    if (j == M - 1) {
      for (int e = tid; e < r * p * cRin; e += nt) W[e] = Min[e];
    } else {  // W[(a u)][c] = sum_b M_j[(a u)][b] L[b][c]
      mgemm64(r * p, cR, cRin, Min, cRin, 1, Lc, cR, 1, W, map1(cR), map1(1), 1.0, tid, nt);
    }
    __syncthreads();
    double* out = env_site(L, ws, z.tmp_slot, j);
    if (j == 0) {
      for (int e = tid; e < p * cR; e += nt) out[e] = W[e];
      __syncthreads();
      break;
    }
    const int c = p * cR, kk = z.chic[j];
    if (NT == 64 && r <= 16 && c <= 128) {  // one wave: W in registers, Q straight to the slot
      lq_wave<16>(W, r, c, out, Ln, bV, tau, tid);
    } else {
      lq_householder(W, r, c, bLW, Ln, bV, tau, rowdot, red, tid, nt);
      for (int e = tid; e < kk * c; e += nt) out[e] = bLW[e];
    }
    for (int e = tid; e < r * kk; e += nt) Lc[e] = Ln[e];
    __syncthreads();
  }

  // ---- phase B: zip left to right.  The carry C[k][l][a] (new bond, the
  // row's bond, the input MPS's bond) and the products below run on the
  // float64 matrix cores in layouts that make every operand single-stride:
  //   Y[(k b)][(l u)] = sum_a       C[(k l)][a] M_j[a][(u b)]
  //   X[(k p)][(b r)] = sum_(l u)   Y[(k b)][(l u)] A[(l u)][(r p)]   (A staged [l][u][r][p])
  double logacc = ws[L.off_envlog + z.in_slot];
  bool near_tie = false;
  if (tid == 0) bC[0] = 1.0;
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, k, j, &dl, &dr, &du, &dd);
    const int Kd = z.nb[j], Ad = z.chic[j], Ld = dl, Rd = dr, Bd = z.chic[j + 1];
    const int Ud = z.dir == 0 ? du : dd, Pd = z.dir == 0 ? dd : du;
    const T4 As = slice(L, k, j, spin(L, k, j));
    const int su = z.dir == 0 ? As.s2 : As.s3, sp = z.dir == 0 ? As.s3 : As.s2;
    const T4 A = stage4(T4{As.p, Ld, Ud, Rd, Pd, As.s0, su, As.s1, sp}, bLW, tid, nt);
    const double* Mg = env_site(L, ws, z.tmp_slot, j);
    double* Mj = bV;
    for (int e = tid; e < Ad * Ud * Bd; e += nt) Mj[e] = Mg[e];
    __syncthreads();
    double* Y = bG;
    mgemm64(Kd * Ld, Ud * Bd, Ad, bC, Ad, 1, Mj, Ud * Bd, 1, Y, map2(Ld, Ud, Bd * Ld * Ud),
            map2(Bd, Ld * Ud, 1), 1.0, tid, nt);
    __syncthreads();
    mgemm64(Kd * Bd, Rd * Pd, Ld * Ud, Y, Ld * Ud, 1, A.p, Rd * Pd, 1, bX,
            map2(Bd, Rd, Pd * Bd * Rd), map2(Pd, Bd * Rd, 1), 1.0, tid, nt);
    __syncthreads();
    const int rows = Kd * Pd, cols = Bd * Rd;
    double* out = env_site(L, ws, z.out_slot, j);
    if (j < M - 1) {
      // sum of |X| (no overflow; NaN and Inf propagate): zero or non-finite X
      double xa = 0.0;
      for (int e = tid; e < rows * cols; e += nt) xa += fabs(bX[e]);
      xa = block_sum(xa, red, tid, nt);
      if (!(xa > 0.0) || !isfinite(xa)) {
        set_flag(ws, L, isfinite(xa) ? kFlagZero : kFlagNonfinite, tid);
        return;
      }
      const int chi = z.nb[j + 1];
      // the carry C is dead until the products after the truncation: its
      // buffer serves as the truncation's small scratch
      top_svd(bX, rows, cols, chi, lam, bUk, bG, bV, bLW, z.lw_doubles, bC, z.c_doubles, z.eig_batch,
              tid, nt);
      const double s1 = lam[0];
      const int nsv = rows < cols ? rows : cols;
      if (chi < nsv) {
        const double sk = lam[chi - 1], sk1 = lam[chi];
        if (sk > kNegligibleRelSv * s1 && (sk - sk1) <= kNearTieRelGap * sk) near_tie = true;
      }
      if (!(s1 > 0.0)) {
        set_flag(ws, L, kFlagZero, tid);
        return;
      }
      for (int e = tid; e < rows * chi; e += nt) {
        const int row = e / chi, c = e - row * chi;
        out[e] = bUk[c * rows + row];
      }
      __syncthreads();
      // C[c][r][b] = sum_row Uk[row][c] X[row][(b r)] / s1
      mgemm64(chi, cols, rows, bUk, rows, 1, bX, cols, 1, bC, map1(cols), map2(Rd, Bd, 1), 1.0 / s1,
              tid, nt);
      __syncthreads();
      logacc += log(s1);
    } else {
      double s = 0.0;
      for (int e = tid; e < rows * cols; e += nt) s += bX[e] * bX[e];
      s = block_sum(s, red, tid, nt);
      const double nrm = sqrt(s);
      if (!(nrm > 0.0) || !isfinite(nrm)) {
        set_flag(ws, L, isfinite(nrm) ? kFlagZero : kFlagNonfinite, tid);
        return;
      }
      for (int e = tid; e < rows * cols; e += nt) out[e] = bX[e] / nrm;
      logacc += log(nrm);
    }
  }
  if (tid == 0) ws[L.off_envlog + z.out_slot] = logacc;
  if (near_tie) set_flag(ws, L, kFlagNearTie, tid);
}

// ---------------------------------------------------------------------------
// k_sandwich
// ---------------------------------------------------------------------------
__device__ inline T3 env_left(const Lat& L, double* ws, int slot, int j, const int* bonds, int ph) {
  if (slot < 0) return T3{L.ones, 1, 1, 1, 0, 0, 0};
  return mps_left(env_site(L, ws, slot, j), bonds[j], ph, bonds[j + 1]);
}
__device__ inline T3 env_right(const Lat& L, double* ws, int slot, int j, const int* bonds, int ph) {
  if (slot < 0) return T3{L.ones, 1, 1, 1, 0, 0, 0};
  return mps_right(env_site(L, ws, slot, j), bonds[j], ph, bonds[j + 1]);
}

template <uint32_t GM>
__global__ void __launch_bounds__(kThreads, 2) k_sandwich(Lat L, SandShape z, BufPlan bp) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  if (sample_dead(ws, L)) return;
  double* gscr = ws + L.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, SB_RED);
  double* bT1 = bufp_t<GM>(bp, lds, gscr, SB_T1);
  double* bT2 = bufp_t<GM>(bp, lds, gscr, SB_T2);
  double* LEa = bufp_t<GM>(bp, lds, gscr, SB_LE0);
  double* LEb = bufp_t<GM>(bp, lds, gscr, SB_LE1);
  double* bE1 = bufp_t<GM>(bp, lds, gscr, SB_E1);
  double* bE2 = bufp_t<GM>(bp, lds, gscr, SB_E2);
  double* bQ = bufp_t<GM>(bp, lds, gscr, SB_Q);
  double* bST = bufp_t<GM>(bp, lds, gscr, SB_STG);
  double* RL = red + kRedDoubles;  // M + 1 log-scales of the right environments
  const int M = L.M, i = z.row;
  const double lsU = z.top_slot < 0 ? 0.0 : ws[L.off_envlog + z.top_slot];
  const double lsD = z.bot_slot < 0 ? 0.0 : ws[L.off_envlog + z.bot_slot];
  double* const re_base = ws + L.off_re;
  const int64_t re_slot = L.re_slot;
#define RE(j) (re_base + (int64_t)(j) * re_slot)

  // right environments RE_j[a][l][b] (left bonds of column j), normalised
  if (tid == 0) {
    RE(M)[0] = 1.0;
    RL[M] = 0.0;
  }
  __syncthreads();
  for (int j = M - 1; j >= 0; --j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_right(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_right(L, ws, z.bot_slot, j, z.tb, dd);
    const T4 A = mirror(slice(L, i, j, spin(L, i, j)));
    update1(RE(j + 1), U, A, Dn, bT1, bT2, RE(j), bST, tid, nt);
    const double lm = normalise(RE(j), z.ta[j] * dl * z.tb[j], red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
    if (tid == 0) RL[j] = RL[j + 1] + lm;
    __syncthreads();
  }
  const double psi_raw = RE(0)[0];
  if (!(psi_raw != 0.0) || !isfinite(psi_raw)) {
    set_flag(ws, L, isfinite(psi_raw) ? kFlagZero : kFlagNonfinite, tid);
    return;
  }
  const double RL0 = RL[0];
  if (tid == 0) {
    ws[L.off_rowlog + i] = RL0 + log(fabs(psi_raw)) + lsU + lsD;
    ws[L.off_rowsign + i] = psi_raw > 0.0 ? 1.0 : -1.0;
  }
  // left sweep: gradients and horizontal ratios
  double* LEc = LEa;
  double* LEn = LEb;
  if (tid == 0) LEc[0] = 1.0;
  __syncthreads();
  double LL = 0.0, eacc = 0.0;
  for (int j = 0; j < M; ++j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_left(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_left(L, ws, z.bot_slot, j, z.tb, dd);
    const uint8_t sj = spin(L, i, j);
    const T4 A = slice(L, i, j, sj);
    upd1_t1(LEc, U, dl, z.tb[j], bT1, bST, tid, nt);
    if (z.want_grad && L.grad) {
      const int Xd = z.ta[j + 1], Bd = z.tb[j], Yd = z.tb[j + 1];
      // Q[(b x)][(r d)] = sum_y Dn[b][d][y] RE_{j+1}[x][r][y]
      const T3 Ds = stage3(Dn, bST, tid, nt);
      __syncthreads();
      mgemm64(Bd * dd, Xd * dr, Yd, Ds.p, Yd, 1, RE(j + 1), 1, Yd, bQ, map2(dd, 1, Xd * dr * dd),
              map2(dr, dd, dr * dd), 1.0, tid, nt);
      __syncthreads();
      // grad[l][r][u][d] = alpha * sum_(b x) T1[(l u)][(b x)] Q[(b x)][(r d)]
      double* go = L.grad + (int64_t)blockIdx.x * L.grad_stride + L.grad_off[i * M + j];
      mgemm64(dl * du, dr * dd, Bd * Xd, bT1, Bd * Xd, 1, bQ, dr * dd, 1, go,
              map2(du, dd, dr * du * dd), map2(dd, 1, du * dd), exp(LL + RL[j + 1] - RL0) / psi_raw,
              tid, nt);
      __syncthreads();
    }
    const bool ratio = z.want_eloc && j < M - 1 && sj != spin(L, i, j + 1);
    if (ratio) {
      const uint8_t sn = spin(L, i, j + 1);
      upd1_rest(bT1, du, z.ta[j + 1], slice(L, i, j, sn), Dn, bT2, bE1, bST, tid, nt);
    }
    if (j < M - 1) upd1_rest(bT1, du, z.ta[j + 1], A, Dn, bT2, LEn, bST, tid, nt);
    if (ratio) {
      int dl2, dr2, du2, dd2;
      site_dims(L.N, L.M, L.D, i, j + 1, &dl2, &dr2, &du2, &dd2);
      const T3 U2 = env_left(L, ws, z.top_slot, j + 1, z.ta, du2);
      const T3 D2 = env_left(L, ws, z.bot_slot, j + 1, z.tb, dd2);
      update1(bE1, U2, slice(L, i, j + 1, sj), D2, bT1, bT2, bE2, bST, tid, nt);
      const double v = dot(bE2, RE(j + 2), z.ta[j + 2] * dr2 * z.tb[j + 2], red, tid, nt);
      const double R = v * exp(LL + RL[j + 2] - RL0) / psi_raw;
      eacc += L.J1 * 0.5 * R;
      if (tid == 0 && L.mbond && L.mbond[blockIdx.x] == i * (M - 1) + j) ws[L.off_flags + 2] = R;
    }
    if (j < M - 1) {
      const double lm = normalise(LEn, z.ta[j + 1] * dr * z.tb[j + 1], red, tid, nt);
      if (!isfinite(lm)) {
        set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
        return;
      }
      LL += lm;
      double* t = LEc;
      LEc = LEn;
      LEn = t;
    }
  }
  if (tid == 0) ws[L.off_eloc] += eacc;
}
#undef RE

// ---------------------------------------------------------------------------
// k_strip
// ---------------------------------------------------------------------------
template <int PREC, uint32_t GM>
__global__ void __launch_bounds__(kThreads, 2) k_strip(Lat L, StripShape z, BufPlan bp) {
  typedef typename PT<PREC>::T T;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  if (sample_dead(ws, L)) return;
  // redo marker: set by a reduced-precision pass whose accuracy check failed
  double* const redo = ws + L.off_flags + 1;
  if (z.refine && *redo == 0.0) return;
  double* gscr = ws + L.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, TB_RED);
  T* bT1 = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_T1));
  T* bT2 = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_T2));
  T* bST = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_STG));
  T* LEa = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_LE0));
  T* LEb = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_LE1));
  T* bE1 = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_E1));
  T* bE2 = reinterpret_cast<T*>(bufp_t<GM>(bp, lds, gscr, TB_E2));
  double* RL = red + kRedDoubles;
  const int M = L.M, i = z.row;
  T* const re2_base = reinterpret_cast<T*>(ws + L.off_re2);
  const int64_t re2_slot = L.re2_slot;
#define RE(j) (re2_base + (int64_t)(j) * re2_slot)

  if (tid == 0) {
    RE(M)[0] = (T)1.0;
    RL[M] = 0.0;
  }
  __syncthreads();
  for (int j = M - 1; j >= 0; --j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    int el, er, eu, ed;
    site_dims(L.N, L.M, L.D, i + 1, j, &el, &er, &eu, &ed);
    const T3 U = env_right(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_right(L, ws, z.bot_slot, j, z.tb, ed);
    const T4 A1 = mirror(slice(L, i, j, spin(L, i, j)));
    const T4 A2 = mirror(slice(L, i + 1, j, spin(L, i + 1, j)));
    update2<PREC>(RE(j + 1), U, A1, A2, Dn, bT1, bT2, RE(j), bST, z.xc, tid, nt);
    const double lm = normalise(RE(j), z.ta[j] * dl * el * z.tb[j], red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
    if (tid == 0) RL[j] = RL[j + 1] + lm;
    __syncthreads();
  }
  const double val0 = (double)RE(0)[0];
  if (!(val0 != 0.0) || !isfinite(val0)) {
    set_flag(ws, L, isfinite(val0) ? kFlagZero : kFlagNonfinite, tid);
    return;
  }
  const double RL0 = RL[0];
  T* LEc = LEa;
  T* LEn = LEb;
  if (tid == 0) LEc[0] = (T)1.0;
  __syncthreads();
  double LL = 0.0, eacc = 0.0;
  double devmax = 0.0, eabs = 0.0;  // reduced precision: accuracy probe and sum of |terms|
  for (int j = 0; j < M; ++j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    int el, er, eu, ed;
    site_dims(L.N, L.M, L.D, i + 1, j, &el, &er, &eu, &ed);
    if constexpr (PREC != 0) {
      // accuracy probe: <LE_j|RE_j> reproduces the strip value at every cut in
      // exact arithmetic; its reduced-precision deviation measures the
      // environments' relative error
      if (j >= 1) {
        const double w = dot(LEc, RE(j), z.ta[j] * dl * el * z.tb[j], red, tid, nt) *
                         exp(LL + RL[j] - RL0) / val0;
        const double dev = fabs(w - 1.0);
        devmax = dev <= devmax ? devmax : (dev == dev ? dev : INFINITY);
        if (!(devmax <= kRefineMaxDev)) break;
      }
    }
    const T3 U = env_left(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_left(L, ws, z.bot_slot, j, z.tb, ed);
    const uint8_t s1 = spin(L, i, j), s2 = spin(L, i + 1, j);
    const T4 A1 = slice(L, i, j, s1), A2 = slice(L, i + 1, j, s2);
    const int nout = z.ta[j + 1] * dr * er * z.tb[j + 1];
    if (s1 != s2) {
      update2<PREC>(LEc, U, slice(L, i, j, s2), slice(L, i + 1, j, s1), Dn, bT1, bT2, bE1, bST, z.xc, tid, nt);
      const double v = dot(bE1, RE(j + 1), nout, red, tid, nt);
      const double R = v * exp(LL + RL[j + 1] - RL0) / val0;
      const double term = L.J1 * 0.5 * R;
      eacc += term;
      eabs += fabs(term);
      if (tid == 0 && L.mbond && L.mbond[blockIdx.x] == L.N * (M - 1) + i * M + j)
        ws[L.off_flags + 2] = R;
    }
    if (z.want_diag && j < M - 1) {
      int fl, fr, fu, fd;
      site_dims(L.N, L.M, L.D, i, j + 1, &fl, &fr, &fu, &fd);
      int gl, gr, gu, gd;
      site_dims(L.N, L.M, L.D, i + 1, j + 1, &gl, &gr, &gu, &gd);
      const T3 U2 = env_left(L, ws, z.top_slot, j + 1, z.ta, fu);
      const T3 D2 = env_left(L, ws, z.bot_slot, j + 1, z.tb, gd);
      const uint8_t c1 = spin(L, i, j + 1), c2 = spin(L, i + 1, j + 1);
      const int n2 = z.ta[j + 2] * fr * gr * z.tb[j + 2];
      if (s1 != c2) {  // (i,j) <-> (i+1,j+1)
        update2<PREC>(LEc, U, slice(L, i, j, c2), A2, Dn, bT1, bT2, bE1, bST, z.xc, tid, nt);
        update2<PREC>(bE1, U2, slice(L, i, j + 1, c1), slice(L, i + 1, j + 1, s1), D2, bT1, bT2,
                bE2, bST, z.xc, tid, nt);
        const double v = dot(bE2, RE(j + 2), n2, red, tid, nt);
        const double term = L.J2 * 0.5 * v * exp(LL + RL[j + 2] - RL0) / val0;
        eacc += term;
        eabs += fabs(term);
      }
      if (c1 != s2) {  // (i,j+1) <-> (i+1,j)
        update2<PREC>(LEc, U, A1, slice(L, i + 1, j, c1), Dn, bT1, bT2, bE1, bST, z.xc, tid, nt);
        update2<PREC>(bE1, U2, slice(L, i, j + 1, s2), slice(L, i + 1, j + 1, c2), D2, bT1, bT2,
                bE2, bST, z.xc, tid, nt);
        const double v = dot(bE2, RE(j + 2), n2, red, tid, nt);
        const double term = L.J2 * 0.5 * v * exp(LL + RL[j + 2] - RL0) / val0;
        eacc += term;
        eabs += fabs(term);
      }
    }
    if (j < M - 1) {
      update2<PREC>(LEc, U, A1, A2, Dn, bT1, bT2, LEn, bST, z.xc, tid, nt);
      const double lm = normalise(LEn, nout, red, tid, nt);
      if (!isfinite(lm)) {
        set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
        return;
      }
      LL += lm;
      T* t = LEc;
      LEc = LEn;
      LEn = t;
    }
  }
  if constexpr (PREC != 0) {
    // estimated energy error of this strip: (environment deviation) x sum |terms|;
    // above the budget the float64 pass recomputes the strip
    const double budget = kRefineTolSite * (double)(L.N * L.M) / (double)(L.N - 1);
    if (!(devmax <= kRefineMaxDev) || !(devmax * eabs <= budget)) {
      if (tid == 0) *redo = 1.0;
      set_flag(ws, L, kFlagRefined, tid);
      return;
    }
  }
  if (tid == 0) {
    ws[L.off_eloc] += eacc;
    if (z.refine) *redo = 0.0;
  }
}
#undef RE

// ---------------------------------------------------------------------------
// Metropolis sweep (the sampling of Sec. II with weight W(S)^2): the
// exchange proposals of one row (horizontal bonds) or one pair of rows
// (vertical bonds), decided in order with u < min(1, R^2).  R is the ratio of
// the two contractions that differ only in the exchanged column(s), taken
// with the same right environments (built once, before the row's proposals)
// and the same left environment, which is extended column by column with the
// spins as they stand after each decision.  The configurations are updated
// in place.  Per sample: uniforms, accepted and ratios hold one entry per bond
// of the sweep, the row's (strip's) bonds from offset k0.
// ---------------------------------------------------------------------------
struct SweepIO {
  uint8_t* cfg;            // the configurations (the same memory as Lat::cfg)
  const double* uniforms;  // [batch][nbonds]
  uint8_t* accepted;       // [batch][nbonds]
  double* ratios;          // [batch][nbonds] or null
  int nbonds;
  int k0;
};

// a spin as it stands during the sweep (read through the configuration the
// sweep writes, never from a cached copy)
__device__ inline uint8_t sweep_spin(const SweepIO& io, const Lat& L, int i, int j) {
  return reinterpret_cast<const volatile uint8_t*>(io.cfg)[(int64_t)blockIdx.x * L.N * L.M +
                                                           i * L.M + j];
}

__device__ inline bool sweep_decide(double num, double den, double u) {
  if (den == 0.0) return num != 0.0;  // leave a zero-weight state at the first nonzero proposal
  const double r = num / den;
  return u < fmin(1.0, r * r);
}

template <uint32_t GM>
__global__ void __launch_bounds__(kThreads, 2) k_sweep_row(Lat L, SandShape z, BufPlan bp,
                                                           SweepIO io) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  if (sample_dead(ws, L)) return;
  double* gscr = ws + L.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, SB_RED);
  double* bT1 = bufp_t<GM>(bp, lds, gscr, SB_T1);
  double* bT2 = bufp_t<GM>(bp, lds, gscr, SB_T2);
  double* bufs[3] = {bufp_t<GM>(bp, lds, gscr, SB_LE0), bufp_t<GM>(bp, lds, gscr, SB_LE1),
                     bufp_t<GM>(bp, lds, gscr, SB_E1)};
  double* bE2 = bufp_t<GM>(bp, lds, gscr, SB_E2);
  double* bST = bufp_t<GM>(bp, lds, gscr, SB_STG);
  const int M = L.M, i = z.row;
  const int64_t b = blockIdx.x;
  double* const re_base = ws + L.off_re;
  const int64_t re_slot = L.re_slot;
#define RE(j) (re_base + (int64_t)(j) * re_slot)
  if (tid == 0) RE(M)[0] = 1.0;
  __syncthreads();
  for (int j = M - 1; j >= 0; --j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_right(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_right(L, ws, z.bot_slot, j, z.tb, dd);
    const T4 A = mirror(slice(L, i, j, spin(L, i, j)));
    update1(RE(j + 1), U, A, Dn, bT1, bT2, RE(j), bST, tid, nt);
    const double lm = normalise(RE(j), z.ta[j] * dl * z.tb[j], red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
  }
  int c = 0;  // bufs[c] holds the left environment of column j
  if (tid == 0) bufs[0][0] = 1.0;
  __syncthreads();
  for (int j = 0; j < M - 1; ++j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_left(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_left(L, ws, z.bot_slot, j, z.tb, dd);
    double* LEc = bufs[c];
    double* Fa = bufs[(c + 1) % 3];
    double* Fb = bufs[(c + 2) % 3];
    const uint8_t sa = sweep_spin(io, L, i, j), sb = sweep_spin(io, L, i, j + 1);
    const int64_t slot = b * io.nbonds + io.k0 + j;
    upd1_t1(LEc, U, dl, z.tb[j], bT1, bST, tid, nt);
    int next;
    if (sa != sb) {
      int dl2, dr2, du2, dd2;
      site_dims(L.N, L.M, L.D, i, j + 1, &dl2, &dr2, &du2, &dd2);
      const T3 U2 = env_left(L, ws, z.top_slot, j + 1, z.ta, du2);
      const T3 D2 = env_left(L, ws, z.bot_slot, j + 1, z.tb, dd2);
      const int n2 = z.ta[j + 2] * dr2 * z.tb[j + 2];
      // exchanged (Fa) and current (Fb) first columns share T1 = LE_j U_j
      upd1_rest(bT1, du, z.ta[j + 1], slice(L, i, j, sb), Dn, bT2, Fa, bST, tid, nt);
      upd1_rest(bT1, du, z.ta[j + 1], slice(L, i, j, sa), Dn, bT2, Fb, bST, tid, nt);
      update1(Fa, U2, slice(L, i, j + 1, sa), D2, bT1, bT2, bE2, bST, tid, nt);
      const double num = dot(bE2, RE(j + 2), n2, red, tid, nt);
      update1(Fb, U2, slice(L, i, j + 1, sb), D2, bT1, bT2, bE2, bST, tid, nt);
      const double den = dot(bE2, RE(j + 2), n2, red, tid, nt);
      const bool ok = sweep_decide(num, den, io.uniforms[slot]);
      if (tid == 0) {
        io.accepted[slot] = ok ? 1 : 0;
        if (io.ratios) io.ratios[slot] = den != 0.0 ? num / den : INFINITY;
        if (ok) {
          io.cfg[b * L.N * M + i * M + j] = sb;
          io.cfg[b * L.N * M + i * M + j + 1] = sa;
        }
      }
      __syncthreads();
      next = ok ? (c + 1) % 3 : (c + 2) % 3;
    } else {
      upd1_rest(bT1, du, z.ta[j + 1], slice(L, i, j, sa), Dn, bT2, Fa, bST, tid, nt);
      next = (c + 1) % 3;
    }
    const double lm = normalise(bufs[next], z.ta[j + 1] * dr * z.tb[j + 1], red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
    c = next;
  }
}
#undef RE

template <uint32_t GM>
__global__ void __launch_bounds__(kThreads, 2) k_sweep_strip(Lat L, StripShape z, BufPlan bp,
                                                             SweepIO io) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  if (sample_dead(ws, L)) return;
  double* gscr = ws + L.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, TB_RED);
  double* bT1 = bufp_t<GM>(bp, lds, gscr, TB_T1);
  double* bT2 = bufp_t<GM>(bp, lds, gscr, TB_T2);
  double* bST = bufp_t<GM>(bp, lds, gscr, TB_STG);
  double* bufs[3] = {bufp_t<GM>(bp, lds, gscr, TB_LE0), bufp_t<GM>(bp, lds, gscr, TB_LE1),
                     bufp_t<GM>(bp, lds, gscr, TB_E1)};
  const int M = L.M, i = z.row;
  const int64_t b = blockIdx.x;
  double* const re2_base = ws + L.off_re2;
  const int64_t re2_slot = L.re2_slot;
#define RE(j) (re2_base + (int64_t)(j) * re2_slot)
  if (tid == 0) RE(M)[0] = 1.0;
  __syncthreads();
  for (int j = M - 1; j >= 0; --j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    int el, er, eu, ed;
    site_dims(L.N, L.M, L.D, i + 1, j, &el, &er, &eu, &ed);
    const T3 U = env_right(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_right(L, ws, z.bot_slot, j, z.tb, ed);
    const T4 A1 = mirror(slice(L, i, j, spin(L, i, j)));
    const T4 A2 = mirror(slice(L, i + 1, j, spin(L, i + 1, j)));
    update2<0>(RE(j + 1), U, A1, A2, Dn, bT1, bT2, RE(j), bST, z.xc, tid, nt);
    const double lm = normalise(RE(j), z.ta[j] * dl * el * z.tb[j], red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
  }
  int c = 0;
  if (tid == 0) bufs[0][0] = 1.0;
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    int dl, dr, du, dd;
    site_dims(L.N, L.M, L.D, i, j, &dl, &dr, &du, &dd);
    int el, er, eu, ed;
    site_dims(L.N, L.M, L.D, i + 1, j, &el, &er, &eu, &ed);
    const T3 U = env_left(L, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_left(L, ws, z.bot_slot, j, z.tb, ed);
    double* LEc = bufs[c];
    double* Fa = bufs[(c + 1) % 3];
    double* Fb = bufs[(c + 2) % 3];
    const uint8_t sa = sweep_spin(io, L, i, j), sb = sweep_spin(io, L, i + 1, j);
    const int nout = z.ta[j + 1] * dr * er * z.tb[j + 1];
    int next;
    if (sa != sb) {
      const int64_t slot = b * io.nbonds + io.k0 + (M - 1) + j;
      update2<0>(LEc, U, slice(L, i, j, sb), slice(L, i + 1, j, sa), Dn, bT1, bT2, Fa, bST,
                 z.xc, tid, nt);
      const double num = dot(Fa, RE(j + 1), nout, red, tid, nt);
      update2<0>(LEc, U, slice(L, i, j, sa), slice(L, i + 1, j, sb), Dn, bT1, bT2, Fb, bST,
                 z.xc, tid, nt);
      const double den = dot(Fb, RE(j + 1), nout, red, tid, nt);
      const bool ok = sweep_decide(num, den, io.uniforms[slot]);
      if (tid == 0) {
        io.accepted[slot] = ok ? 1 : 0;
        if (io.ratios) io.ratios[slot] = den != 0.0 ? num / den : INFINITY;
        if (ok) {
          io.cfg[b * L.N * M + i * M + j] = sb;
          io.cfg[b * L.N * M + (i + 1) * M + j] = sa;
        }
      }
      __syncthreads();
      next = ok ? (c + 1) % 3 : (c + 2) % 3;
    } else {
      if (j == M - 1) break;
      update2<0>(LEc, U, slice(L, i, j, sa), slice(L, i + 1, j, sb), Dn, bT1, bT2, Fa, bST,
                 z.xc, tid, nt);
      next = (c + 1) % 3;
    }
    if (j == M - 1) break;
    const double lm = normalise(bufs[next], nout, red, tid, nt);
    if (!isfinite(lm)) {
      set_flag(ws, L, isnan(lm) ? kFlagNonfinite : kFlagZero, tid);
      return;
    }
    c = next;
  }
}
#undef RE

// zero the accepted flags and set the ratios to NaN before a sweep (one
// thread per entry)
__global__ void __launch_bounds__(kThreads) k_sweep_clear(int64_t n, uint8_t* accepted,
                                                          double* ratios) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  accepted[q] = 0;
  if (ratios) ratios[q] = NAN;
}

// ---------------------------------------------------------------------------
// k_metropolis: one exchange proposal per sample, decided from the ratio its
// evaluation already holds (one thread per sample)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_metropolis(Lat L, int nb, const double* uniforms,
                                                         uint8_t* cfg, uint8_t* accepted) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double* ws = L.ws + (int64_t)b * L.ws_stride;
  const int N = L.N, M = L.M, nh = N * (M - 1), nbonds = nh + (N - 1) * M;
  const int bond = L.mbond[b];
  uint8_t acc = 0;
  const uint32_t f = *reinterpret_cast<const uint32_t*>(ws + L.off_flags);
  if (bond >= 0 && bond < nbonds && !(f & (kFlagZero | kFlagNonfinite))) {
    int sa, sb;
    if (bond < nh) {
      sa = (bond / (M - 1)) * M + bond % (M - 1);
      sb = sa + 1;
    } else {
      sa = bond - nh;
      sb = sa + M;
    }
    uint8_t* c = cfg + (int64_t)b * N * M;
    if (c[sa] != c[sb]) {
      const double R = ws[L.off_flags + 2];
      if (isfinite(R) && uniforms[b] < fmin(1.0, R * R)) {
        const uint8_t t = c[sa];
        c[sa] = c[sb];
        c[sb] = t;
        acc = 1;
      }
    }
  }
  accepted[b] = acc;
}

// ---------------------------------------------------------------------------
// Gradient optimisation, Eqs. (3) and (6): per-element sums over samples of
// Delta and Delta E (Delta of a sample belongs to the slice of its spin), the
// scalar sums n, sum E, sum E^2, and the sign update of the tensors.
// ---------------------------------------------------------------------------
struct GoArgs {
  int batch, nsites, gel;
  int64_t grad_stride;       // doubles from one sample's Delta block to the next (>= gel)
  const uint8_t* cfg;        // [batch][nsites]
  const double* grad;        // [batch][grad_stride], the first gel of each row used
  const double* eloc;        // [batch]
  const uint32_t* flags;     // [batch]
  const int64_t* grad_off;   // [nsites] first gradient element of each site
  const int64_t* site_off;   // [nsites] first tensor element of each site
  double* sd;                // tensor-shaped sums of Delta
  double* sde;               // tensor-shaped sums of Delta E
};

// one thread per gradient element (site k, slice entry e), both spins
__global__ void __launch_bounds__(kThreads) k_go_accumulate(GoArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.gel) return;
  int lo = 0, hi = a.nsites - 1;  // the site whose block holds g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.grad_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int64_t blk = (k + 1 < a.nsites ? a.grad_off[k + 1] : a.gel) - a.grad_off[k];
  const int64_t e = g - a.grad_off[k];
  // eight samples per step with independent loads (more bytes in flight per
  // wave); partial sums per lane of the step, combined in a fixed order at the
  // end, so the result does not depend on timing
  constexpr int U = 8;
  double s0[U], s1[U], t0[U], t1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) s0[u] = s1[u] = t0[u] = t1[u] = 0.0;
  const int bfull = a.batch - a.batch % U;
  for (int b = 0; b < bfull; b += U) {
    double d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) d[u] = a.grad[(int64_t)(b + u) * a.grad_stride + g];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = !(a.flags[b + u] & (kFlagZero | kFlagNonfinite));
      const bool up = a.cfg[(int64_t)(b + u) * a.nsites + k] != 0;
      const double v = ok ? d[u] : 0.0, ve = ok ? d[u] * a.eloc[b + u] : 0.0;
      s1[u] += up ? v : 0.0;
      t1[u] += up ? ve : 0.0;
      s0[u] += up ? 0.0 : v;
      t0[u] += up ? 0.0 : ve;
    }
  }
  for (int b = bfull; b < a.batch; ++b) {
    if (a.flags[b] & (kFlagZero | kFlagNonfinite)) continue;
    const double d = a.grad[(int64_t)b * a.grad_stride + g];
    const double de = d * a.eloc[b];
    if (a.cfg[(int64_t)b * a.nsites + k]) {
      s1[0] += d;
      t1[0] += de;
    } else {
      s0[0] += d;
      t0[0] += de;
    }
  }
#pragma unroll
  for (int u = 1; u < U; ++u) {
    s0[0] += s0[u];
    s1[0] += s1[u];
    t0[0] += t0[u];
    t1[0] += t1[u];
  }
  const int64_t q0 = a.site_off[k] + e, q1 = q0 + blk;
  a.sd[q0] += s0[0];
  a.sd[q1] += s1[0];
  a.sde[q0] += t0[0];
  a.sde[q1] += t1[0];
}

// stats[0..2] += (n, sum E, sum E^2) over the unflagged samples (one workgroup)
__global__ void __launch_bounds__(kThreads) k_go_stats(int batch, const double* eloc,
                                                       const uint32_t* flags, double* stats) {
  __shared__ double red[kRedDoubles];
  const int tid = threadIdx.x, nt = blockDim.x;
  double n = 0.0, se = 0.0, se2 = 0.0;
  for (int b = tid; b < batch; b += nt) {
    if (flags[b] & (kFlagZero | kFlagNonfinite)) continue;
    n += 1.0;
    se += eloc[b];
    se2 += eloc[b] * eloc[b];
  }
  n = block_sum(n, red, tid, nt);
  se = block_sum(se, red, tid, nt);
  se2 = block_sum(se2, red, tid, nt);
  if (tid == 0) {
    stats[0] += n;
    stats[1] += se;
    stats[2] += se2;
  }
}

// T -= p dt sign(2 <Delta E> - 2 <Delta><E>), element by element
__global__ void __launch_bounds__(kThreads) k_go_update(int64_t nparams, double* T,
                                                        const double* sd, const double* sde,
                                                        const double* stats, double dt,
                                                        const double* p) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nparams) return;
  const double n = stats[0];
  if (!(n > 0.0)) return;
  const double g = 2.0 * sde[q] / n - 2.0 * (sd[q] / n) * (stats[1] / n);
  const double sg = g > 0.0 ? 1.0 : (g < 0.0 ? -1.0 : 0.0);
  T[q] -= p[q] * dt * sg;
}

// ---------------------------------------------------------------------------
// Spin-spin correlations on a window of the lattice (Sec. IV): per pair of
// window sites, the number of samples whose two spins are equal.  Integer
// counts, so the result does not depend on the order of the additions.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_sz_counts(int M, int r0, int c0, int w, int nw,
                                                        int nsites, int batch, int chunk,
                                                        const uint8_t* cfg, const uint32_t* flags,
                                                        unsigned long long* same,
                                                        unsigned long long* nsamples) {
  const int pair = blockIdx.x * blockDim.x + threadIdx.x;
  const int b0 = blockIdx.y * chunk, b1 = min(batch, b0 + chunk);
  if (pair >= nw * nw) return;
  const int p = pair / nw, q = pair % nw;
  const int sp = (r0 + p / w) * M + c0 + p % w, sq = (r0 + q / w) * M + c0 + q % w;
  unsigned long long cnt = 0, n = 0;
  for (int b = b0; b < b1; ++b) {
    if (flags && (flags[b] & (kFlagZero | kFlagNonfinite))) continue;
    const uint8_t* s = cfg + (int64_t)b * nsites;
    cnt += s[sp] == s[sq] ? 1ull : 0ull;
    ++n;
  }
  if (cnt) atomicAdd(same + pair, cnt);
  if (pair == 0 && n) atomicAdd(nsamples, n);
}

// factor / Nw^2 * sum_ij C_ij cos(k.(r_i - r_j)), one workgroup, with
// C_ij = <S^z_i S^z_j>, plus the transverse average trans_ij / ntrans[0] when
// trans is given (C_ij = <S_i . S_j>)
__global__ void __launch_bounds__(kThreads) k_structure_factor(int h, int w, const unsigned long long* same,
                                                               const unsigned long long* nsamples,
                                                               const double* trans,
                                                               const int64_t* ntrans, double kx,
                                                               double ky, double factor, double* out) {
  __shared__ double red[kRedDoubles];
  const int tid = threadIdx.x, nt = blockDim.x, nw = h * w;
  const double n = (double)nsamples[0];
  const double m = trans ? (double)ntrans[0] : 1.0;
  double acc = 0.0;
  for (int pair = tid; pair < nw * nw; pair += nt) {
    const int p = pair / nw, q = pair % nw;
    double c = (2.0 * (double)same[pair] - n) / (4.0 * n);
    if (trans) c += trans[pair] / m;
    acc += c * cos(kx * (double)(p % w - q % w) + ky * (double)(p / w - q / w));
  }
  acc = block_sum(acc, red, tid, nt);
  if (tid == 0) out[0] = n > 0.0 && m > 0.0 ? factor * acc / ((double)nw * nw) : __builtin_nan("");
}

// ---------------------------------------------------------------------------
// Transverse correlations (Sec. IV): exchange ratios W(S^{pq})/W(S) for every
// pair of window sites p before q (row-major) with s_p != s_q.  For p in row
// a and q in row b >= a both contractions share U_{a-1}(S) and Dn_{b+1}(S):
// the numerator zips rows a..b-1 of S^{pq} into U_{a-1}(S) and closes with the
// exact row-b sandwich; the denominator is psi_b(S).
//
// One instance per (window site p, sample r), instance v = x * nbr + r with x
// the window index of p, so the instances whose p lies in the first k window
// rows form the prefix [0, k w nbr) of the instance batch.  An instance
// evaluates S_r with the spin at p flipped (S^p): its top chain starts from a
// copy of U_{a-1}(S_r); at each row b >= a one pass gives, for every window
// column c, psi_b(S^p with (b, c) flipped as well) = psi_b(S^{pq}), since
// exchanging two unequal spins flips both.
// ---------------------------------------------------------------------------

// instance configurations, cleared flags and log-scales, ratio rows set to NaN
__global__ void __launch_bounds__(kThreads) k_corr_init(Lat V, FlipShape z, const uint8_t* cfg_real,
                                                        uint8_t* cfg_inst) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int v = blockIdx.x, x = v / z.nbr, r = v - x * z.nbr;
  const int ns = V.N * V.M, n = z.h * z.w;
  const int p = (z.r0 + x / z.w) * V.M + z.c0 + x % z.w;
  const uint8_t* src = cfg_real + (int64_t)r * ns;
  uint8_t* dst = cfg_inst + (int64_t)v * ns;
  for (int k = tid; k < ns; k += nt) dst[k] = k == p ? (uint8_t)(1 - src[k]) : src[k];
  double* ws = V.ws + (int64_t)v * V.ws_stride;
  for (int e = tid; e < n; e += nt) ws[z.off_rat + e] = __builtin_nan("");
  if (tid == 0) {
    *reinterpret_cast<uint32_t*>(ws + V.off_flags) = 0u;
    for (int q = 0; q < 3; ++q) ws[V.off_envlog + q] = 0.0;
  }
}

// U_{a-1}(S_r) into the top slot of the instances [v0, v0 + count) (their p in
// row a); an instance of a sample already stopped (zero or non-finite) stops too
__global__ void __launch_bounds__(kThreads) k_corr_copy(Lat V, Lat R, int nbr, int v0, int src_slot,
                                                        int dst_slot) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int v = v0 + blockIdx.x, r = v % nbr;
  const double* wr = R.ws + (int64_t)r * R.ws_stride;
  double* wv = V.ws + (int64_t)v * V.ws_stride;
  const double* a = wr + R.off_env + (int64_t)src_slot * R.env_stride;
  double* b = wv + V.off_env + (int64_t)dst_slot * V.env_stride;
  for (int64_t e = tid; e < R.env_stride; e += nt) b[e] = a[e];
  if (tid == 0) {
    wv[V.off_envlog + dst_slot] = wr[R.off_envlog + src_slot];
    const uint32_t f = *reinterpret_cast<const uint32_t*>(wr + R.off_flags);
    *reinterpret_cast<uint32_t*>(wv + V.off_flags) |= f & (kFlagZero | kFlagNonfinite);
  }
}

// Row z.row of every instance of the prefix: right environments of S^p, then a
// left sweep that closes, at each window column c of the row whose pair with p
// is counted here, the column with the other spin slice:
//   R_pq = <LE_c| col c flipped |RE_{c+1}> * (log-scales) / psi_b(S_r).
template <uint32_t GM>
__global__ void __launch_bounds__(kThreads, 2) k_flip_row(Lat V, Lat R, FlipShape z, BufPlan bp) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int v = blockIdx.x, x = v / z.nbr, r = v - x * z.nbr;
  double* ws = V.ws + (int64_t)v * V.ws_stride;
  double* wr = R.ws + (int64_t)r * R.ws_stride;
  const int M = V.M, i = z.row;
  const int ap = z.r0 + x / z.w, cp = z.c0 + x % z.w;
  const int y0 = (i - z.r0) * z.w - z.c0;  // window index of (i, c) is y0 + c
  const uint8_t sflip = spin(V, ap, cp);   // 1 - s_p: the spin a counted partner q has
  double* rat = ws + z.off_rat;
  const uint32_t f = *reinterpret_cast<const uint32_t*>(ws + V.off_flags);
  if (f & kFlagNonfinite) return;
  if (f & kFlagZero) {  // the chain above this row vanished: every such W(S^{pq}) is 0
    for (int c = z.c0 + tid; c < z.c0 + z.w; c += nt)
      if (y0 + c > x && spin(V, i, c) == sflip) rat[y0 + c] = 0.0;
    return;
  }
  double* gscr = ws + V.off_scratch;
  double* red = bufp_t<GM>(bp, lds, gscr, SB_RED);
  double* bT1 = bufp_t<GM>(bp, lds, gscr, SB_T1);
  double* bT2 = bufp_t<GM>(bp, lds, gscr, SB_T2);
  double* LEa = bufp_t<GM>(bp, lds, gscr, SB_LE0);
  double* LEb = bufp_t<GM>(bp, lds, gscr, SB_LE1);
  double* bE1 = bufp_t<GM>(bp, lds, gscr, SB_E1);
  double* bST = bufp_t<GM>(bp, lds, gscr, SB_STG);
  double* RL = red + kRedDoubles;
  const double lsU = z.top_slot < 0 ? 0.0 : ws[V.off_envlog + z.top_slot];
  const double lsD = z.bot_slot < 0 ? 0.0 : wr[R.off_envlog + z.bot_slot];
  const double den_log = wr[R.off_rowlog + i], den_sign = wr[R.off_rowsign + i];
  double* const re_base = ws + V.off_re;
  const int64_t re_slot = V.re_slot;
#define RE(j) (re_base + (int64_t)(j) * re_slot)
  // right environments up to the first window column (zero ones stay zero,
  // with log-scale -inf: the values they close are then exactly 0)
  if (tid == 0) {
    RE(M)[0] = 1.0;
    RL[M] = 0.0;
  }
  __syncthreads();
  for (int j = M - 1; j >= z.c0; --j) {
    int dl, dr, du, dd;
    site_dims(V.N, V.M, V.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_right(V, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_right(R, wr, z.bot_slot, j, z.tb, dd);
    const T4 A = mirror(slice(V, i, j, spin(V, i, j)));
    update1(RE(j + 1), U, A, Dn, bT1, bT2, RE(j), bST, tid, nt);
    const double lm = normalise(RE(j), z.ta[j] * dl * z.tb[j], red, tid, nt);
    if (lm != lm) {
      set_flag(ws, V, kFlagNonfinite, tid);
      return;
    }
    if (tid == 0) RL[j] = RL[j + 1] + lm;
    __syncthreads();
  }
  double* LEc = LEa;
  double* LEn = LEb;
  if (tid == 0) LEc[0] = 1.0;
  __syncthreads();
  double LL = 0.0;
  const int cend = z.c0 + z.w;  // columns beyond the window are not needed
  for (int j = 0; j < cend; ++j) {
    int dl, dr, du, dd;
    site_dims(V.N, V.M, V.D, i, j, &dl, &dr, &du, &dd);
    const T3 U = env_left(V, ws, z.top_slot, j, z.ta, du);
    const T3 Dn = env_left(R, wr, z.bot_slot, j, z.tb, dd);
    const uint8_t sj = spin(V, i, j);
    upd1_t1(LEc, U, dl, z.tb[j], bT1, bST, tid, nt);
    if (j >= z.c0 && y0 + j > x && sj == sflip) {
      upd1_rest(bT1, du, z.ta[j + 1], slice(V, i, j, 1 - sj), Dn, bT2, bE1, bST, tid, nt);
      const double val = dot(bE1, RE(j + 1), z.ta[j + 1] * dr * z.tb[j + 1], red, tid, nt);
      if (tid == 0)
        rat[y0 + j] = val == 0.0 ? 0.0
                                 : val * den_sign * exp(LL + RL[j + 1] + lsU + lsD - den_log);
    }
    if (j < cend - 1) {
      upd1_rest(bT1, du, z.ta[j + 1], slice(V, i, j, sj), Dn, bT2, LEn, bST, tid, nt);
      const double lm = normalise(LEn, z.ta[j + 1] * dr * z.tb[j + 1], red, tid, nt);
      if (lm != lm) {
        set_flag(ws, V, kFlagNonfinite, tid);
        return;
      }
      LL += lm;
      double* t = LEc;
      LEc = LEn;
      LEn = t;
    }
  }
#undef RE
}

// Per sample: its flags (the sample's own, NEAR_TIE when a zip of one of its
// instances met a near tie, NONFINITE when a counted ratio is not finite) and,
// when asked, its ratio matrix [n][n] (NaN on the diagonal and where s_p = s_q).
__global__ void __launch_bounds__(kThreads) k_corr_finish(Lat V, Lat R, FlipShape z,
                                                          uint32_t* flags, double* ratios) {
  __shared__ double red[kRedDoubles];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r = blockIdx.x, n = z.h * z.w, M = R.M;
  const double* wr = R.ws + (int64_t)r * R.ws_stride;
  const uint8_t* s = R.cfg + (int64_t)r * R.N * M;
  uint32_t f = *reinterpret_cast<const uint32_t*>(wr + R.off_flags);
  const bool dead = (f & (kFlagZero | kFlagNonfinite)) != 0;
  double tie = 0.0, bad = 0.0;
  for (int x = tid; x < n; x += nt) {
    const double* wv = V.ws + ((int64_t)x * z.nbr + r) * V.ws_stride;
    if (*reinterpret_cast<const uint32_t*>(wv + V.off_flags) & kFlagNearTie) tie = 1.0;
  }
  for (int e = tid; e < n * n; e += nt) {
    const int x = e / n, y = e - x * n;
    const int p = (z.r0 + x / z.w) * M + z.c0 + x % z.w;
    const int q = (z.r0 + y / z.w) * M + z.c0 + y % z.w;
    double val = __builtin_nan("");
    if (!dead && x != y && s[p] != s[q]) {
      const int lo = x < y ? x : y, hi = x < y ? y : x;
      val = V.ws[((int64_t)lo * z.nbr + r) * V.ws_stride + z.off_rat + hi];
      if (!isfinite(val)) bad = 1.0;
    }
    if (ratios) ratios[(int64_t)r * n * n + e] = val;
  }
  tie = block_max(tie, red, tid, nt);
  bad = block_max(bad, red, tid, nt);
  if (tid == 0) {
    if (tie > 0.0) f |= kFlagNearTie;
    if (bad > 0.0) f |= kFlagNonfinite;
    flags[r] = f;
  }
}

// sums[x n + y] += sum over the chunk's counted samples of O_xy (1/2 R_xy for
// a counted pair, 1/2 on the diagonal); count[0] += counted samples.  One
// thread per pair adds the samples one by one, in order, to the running sum:
// the result depends neither on timing nor on how the batch was chunked.
__global__ void __launch_bounds__(kThreads) k_corr_sums(Lat V, Lat R, FlipShape z,
                                                        const uint32_t* flags, double* sums,
                                                        int64_t* count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = z.h * z.w, M = R.M;
  if (e >= n * n) return;
  const int x = e / n, y = e - x * n;
  const int p = (z.r0 + x / z.w) * M + z.c0 + x % z.w;
  const int q = (z.r0 + y / z.w) * M + z.c0 + y % z.w;
  const int lo = x < y ? x : y, hi = x < y ? y : x;
  double acc = sums[e];
  int64_t cnt = 0;
  for (int r = 0; r < z.nbr; ++r) {
    if (flags[r] & (kFlagZero | kFlagNonfinite)) continue;
    ++cnt;
    if (x == y) {
      acc += 0.5;
    } else {
      const uint8_t* s = R.cfg + (int64_t)r * R.N * M;
      if (s[p] != s[q]) acc += 0.5 * V.ws[((int64_t)lo * z.nbr + r) * V.ws_stride + z.off_rat + hi];
    }
  }
  sums[e] = acc;
  if (e == 0) count[0] += cnt;
}

// ---------------------------------------------------------------------------
// k_finalize
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_finalize(Lat L, int want_eloc, double* logabs,
                                                       int8_t* sign, double* eloc,
                                                       uint32_t* flags) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double* ws = sample_ws(L);
  const int b = blockIdx.x;
  uint32_t f = *reinterpret_cast<uint32_t*>(ws + L.off_flags);
  double la = -INFINITY, e = NAN;
  int sg = 0;
  if (!(f & (kFlagZero | kFlagNonfinite))) {
    la = ws[L.off_rowlog + L.N - 1];
    sg = ws[L.off_rowsign + L.N - 1] > 0.0 ? 1 : -1;
    if (want_eloc) {
      // diagonal part: J Sz_a Sz_b over all pairs, Sz = 1/2 - s
      int nn = 0, nnn = 0;  // (#parallel - #antiparallel) per kind
      for (int i = 0; i < L.N; ++i)
        for (int j = 0; j < L.M; ++j) {
          const int s = spin(L, i, j);
          if (j + 1 < L.M) nn += (s == spin(L, i, j + 1)) ? 1 : -1;
          if (i + 1 < L.N) {
            nn += (s == spin(L, i + 1, j)) ? 1 : -1;
            if (j + 1 < L.M) {
              nnn += (s == spin(L, i + 1, j + 1)) ? 1 : -1;
              nnn += (spin(L, i, j + 1) == spin(L, i + 1, j)) ? 1 : -1;
            }
          }
        }
      e = 0.25 * (L.J1 * nn + L.J2 * nnn) + ws[L.off_eloc];
    }
    if (!isfinite(la) || (want_eloc && !isfinite(e))) f |= kFlagNonfinite;
  }
  const bool dead = (f & (kFlagZero | kFlagNonfinite)) != 0;
  if (dead) {
    la = (f & kFlagZero) ? -INFINITY : NAN;
    sg = 0;
    e = NAN;
    if (L.grad) {
      double* g = L.grad + (int64_t)b * L.grad_stride;
      for (int q = tid; q < L.grad_stride; q += nt) g[q] = NAN;
    }
  }
  if (tid == 0) {
    logabs[b] = la;
    sign[b] = (int8_t)sg;
    eloc[b] = e;
    flags[b] = f;
  }
}

// ---------------------------------------------------------------------------
// Workspace of pepsgo_evaluate_noalloc: a fixed array in device memory (each
// device that loads the library holds one until the process ends).  Host code
// must not pass `scratch` itself to a kernel: in host code the name stands
// for a host-side symbol, not a device address.  scratch_address() returns
// the device address on the current device; every use goes through it.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PEPSGO_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_address(void** ptr) {
  *ptr = nullptr;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_edges(const Lat& L, int nb, int slot_top0, int slot_bot, int reset,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_edges, dim3(nb), dim3(kThreads), 0, s, L, slot_top0, slot_bot, reset);
  return hipGetLastError();
}

// Raise a kernel's dynamic LDS limit once to the largest size requested so
// far (launches inside a stream capture then make no attribute calls once
// the sizes were prepared beforehand).
static hipError_t set_lds(const void* fn, int bytes) {
  if (bytes <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::map<const void*, int> done;
  std::lock_guard<std::mutex> g(mu);
  int& have = done[fn];
  if (have >= bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) have = bytes;
  return e;
}

template <uint32_t GM, int NT>
static hipError_t launch_zip_g(const Lat& L, const ZipShape& z, const BufPlan& p, int lds, int nb,
                               hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_zip<GM, NT>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zip<GM, NT>), dim3(nb), dim3(NT), lds, s, L, z, p);
  return hipGetLastError();
}

// placements with a compiled specialisation; any other plan runs the
// run-time variant.  Four-wave workgroups: X in the workspace (the usual
// plan) or everything in LDS.  One-wave workgroups (about 20 KB of LDS):
// work arrays and vectors in LDS, the rest in the workspace.
constexpr uint32_t kZipW1 = (1u << ZB_G) | (1u << ZB_LW) | (1u << ZB_X);
constexpr uint32_t kZipW2 = (1u << ZB_G) | (1u << ZB_LW);
hipError_t launch_zip(const Lat& L, const ZipShape& z, const BufPlan& p, int lds, int nb,
                      hipStream_t s) {
  if (z.threads == 64) {
    if (p.glob == kZipW1) return launch_zip_g<kZipW1, 64>(L, z, p, lds, nb, s);
    if (p.glob == kZipW2) return launch_zip_g<kZipW2, 64>(L, z, p, lds, nb, s);
    return launch_zip_g<kGlobAny, 64>(L, z, p, lds, nb, s);
  }
  if (p.glob == (1u << ZB_X)) return launch_zip_g<(1u << ZB_X), 256>(L, z, p, lds, nb, s);
  if (p.glob == 0u) return launch_zip_g<0u, 256>(L, z, p, lds, nb, s);
  return launch_zip_g<kGlobAny, 256>(L, z, p, lds, nb, s);
}

// Buffer placements with compiled specialisations (glob masks); any other
// plan runs the run-time variant.
constexpr uint32_t kSandQ = 1u << SB_Q;                                    // full LDS budget
constexpr uint32_t kSandT2E2Q = (1u << SB_T2) | (1u << SB_E2) | (1u << SB_Q);  // 80 KB
constexpr uint32_t kStripLE = (1u << TB_LE0) | (1u << TB_LE1) | (1u << TB_E1) | (1u << TB_E2);
constexpr uint32_t kStripE = (1u << TB_E1) | (1u << TB_E2);

template <uint32_t GM>
static hipError_t launch_sandwich_g(const Lat& L, const SandShape& z, const BufPlan& p, int lds,
                                    int nb, hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_sandwich<GM>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sandwich<GM>, dim3(nb), dim3(kThreads), lds, s, L, z, p);
  return hipGetLastError();
}

hipError_t launch_sandwich(const Lat& L, const SandShape& z, const BufPlan& p, int lds, int nb,
                           hipStream_t s) {
  if (p.glob == kSandQ) return launch_sandwich_g<kSandQ>(L, z, p, lds, nb, s);
  if (p.glob == kSandT2E2Q) return launch_sandwich_g<kSandT2E2Q>(L, z, p, lds, nb, s);
  return launch_sandwich_g<kGlobAny>(L, z, p, lds, nb, s);
}

template <int PREC, uint32_t GM>
static hipError_t launch_strip_g(const Lat& L, const StripShape& z, const BufPlan& p, int lds,
                                 int nb, hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_strip<PREC, GM>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_strip<PREC, GM>), dim3(nb), dim3(kThreads), lds, s, L, z, p);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_strip_p(const Lat& L, const StripShape& z, const BufPlan& p, int lds,
                                 int nb, hipStream_t s) {
  if (p.glob == kStripLE) return launch_strip_g<PREC, kStripLE>(L, z, p, lds, nb, s);
  if constexpr (PREC == 1)
    if (p.glob == kStripE) return launch_strip_g<PREC, kStripE>(L, z, p, lds, nb, s);
  return launch_strip_g<PREC, kGlobAny>(L, z, p, lds, nb, s);
}

hipError_t launch_strip(const Lat& L, const StripShape& z, const BufPlan& p, int lds, int nb,
                        int precision, hipStream_t s) {
  if (precision == PEPSGO_FP32) return launch_strip_p<1>(L, z, p, lds, nb, s);
  if (precision == PEPSGO_BF16_MIXED) return launch_strip_p<2>(L, z, p, lds, nb, s);
  if (precision == PEPSGO_BF16) return launch_strip_p<3>(L, z, p, lds, nb, s);
  return launch_strip_p<0>(L, z, p, lds, nb, s);
}

template <uint32_t GM>
static hipError_t launch_sweep_row_g(const Lat& L, const SandShape& z, const BufPlan& p, int lds,
                                     int nb, const SweepIO& io, hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_sweep_row<GM>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sweep_row<GM>, dim3(nb), dim3(kThreads), lds, s, L, z, p, io);
  return hipGetLastError();
}

hipError_t launch_sweep_row(const Lat& L, const SandShape& z, const BufPlan& p, int lds, int nb,
                            uint8_t* cfg, const double* uniforms, uint8_t* accepted,
                            double* ratios, int nbonds, int k0, hipStream_t s) {
  const SweepIO io{cfg, uniforms, accepted, ratios, nbonds, k0};
  if (p.glob == kSandQ) return launch_sweep_row_g<kSandQ>(L, z, p, lds, nb, io, s);
  if (p.glob == kSandT2E2Q) return launch_sweep_row_g<kSandT2E2Q>(L, z, p, lds, nb, io, s);
  return launch_sweep_row_g<kGlobAny>(L, z, p, lds, nb, io, s);
}

template <uint32_t GM>
static hipError_t launch_sweep_strip_g(const Lat& L, const StripShape& z, const BufPlan& p,
                                       int lds, int nb, const SweepIO& io, hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_sweep_strip<GM>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sweep_strip<GM>, dim3(nb), dim3(kThreads), lds, s, L, z, p, io);
  return hipGetLastError();
}

hipError_t launch_sweep_strip(const Lat& L, const StripShape& z, const BufPlan& p, int lds,
                              int nb, uint8_t* cfg, const double* uniforms, uint8_t* accepted,
                              double* ratios, int nbonds, int k0, hipStream_t s) {
  const SweepIO io{cfg, uniforms, accepted, ratios, nbonds, k0};
  if (p.glob == kStripLE) return launch_sweep_strip_g<kStripLE>(L, z, p, lds, nb, io, s);
  return launch_sweep_strip_g<kGlobAny>(L, z, p, lds, nb, io, s);
}

hipError_t launch_sweep_clear(int64_t n, uint8_t* accepted, double* ratios, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_clear, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, n, accepted, ratios);
  return hipGetLastError();
}

// Set the LDS limits of every variant a plan with these sizes may launch (for
// stream capture, which must make no attribute calls).
hipError_t prepare_lds(int lds_zip, int lds_sand, int lds_strip, int precision) {
  const void* fz[] = {reinterpret_cast<const void*>(&k_zip<(1u << ZB_X), 256>),
                      reinterpret_cast<const void*>(&k_zip<0u, 256>),
                      reinterpret_cast<const void*>(&k_zip<kGlobAny, 256>),
                      reinterpret_cast<const void*>(&k_zip<kZipW1, 64>),
                      reinterpret_cast<const void*>(&k_zip<kZipW2, 64>),
                      reinterpret_cast<const void*>(&k_zip<kGlobAny, 64>)};
  const void* fs[] = {reinterpret_cast<const void*>(&k_sandwich<kSandQ>),
                      reinterpret_cast<const void*>(&k_sandwich<kSandT2E2Q>),
                      reinterpret_cast<const void*>(&k_sandwich<kGlobAny>)};
  const void* ft[3];
  int nft = 2;
  if (precision == PEPSGO_FP32) {
    ft[0] = reinterpret_cast<const void*>(&k_strip<1, kStripLE>);
    ft[1] = reinterpret_cast<const void*>(&k_strip<1, kGlobAny>);
    ft[2] = reinterpret_cast<const void*>(&k_strip<1, kStripE>);
    nft = 3;
  } else if (precision == PEPSGO_BF16_MIXED) {
    ft[0] = reinterpret_cast<const void*>(&k_strip<2, kStripLE>);
    ft[1] = reinterpret_cast<const void*>(&k_strip<2, kGlobAny>);
  } else if (precision == PEPSGO_BF16) {
    ft[0] = reinterpret_cast<const void*>(&k_strip<3, kStripLE>);
    ft[1] = reinterpret_cast<const void*>(&k_strip<3, kGlobAny>);
  } else {
    ft[0] = reinterpret_cast<const void*>(&k_strip<0, kStripLE>);
    ft[1] = reinterpret_cast<const void*>(&k_strip<0, kGlobAny>);
  }
  hipError_t e = hipSuccess;
  for (const void* f : fz)
    if (e == hipSuccess) e = set_lds(f, lds_zip);
  for (const void* f : fs)
    if (e == hipSuccess) e = set_lds(f, lds_sand);
  for (int q = 0; q < nft; ++q)
    if (e == hipSuccess) e = set_lds(ft[q], lds_strip);
  return e;
}

hipError_t launch_go_accumulate(int batch, int nsites, int64_t gel, int64_t grad_stride,
                                const uint8_t* cfg, const double* grad, const double* eloc,
                                const uint32_t* flags, const int64_t* grad_off,
                                const int64_t* site_off, double* sd, double* sde, double* stats,
                                hipStream_t s) {
  GoArgs a{batch, nsites, (int)gel, grad_stride, cfg, grad, eloc, flags, grad_off, site_off, sd, sde};
  hipLaunchKernelGGL(k_go_accumulate, dim3((unsigned)((gel + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_go_stats, dim3(1), dim3(kThreads), 0, s, batch, eloc, flags, stats);
  return hipGetLastError();
}

hipError_t launch_sz_counts(int N, int M, int r0, int c0, int h, int w, int batch,
                            const uint8_t* cfg, const uint32_t* flags, int64_t* same,
                            int64_t* nsamples, hipStream_t s) {
  const int nw = h * w, chunk = 2048;
  dim3 grid((unsigned)((nw * nw + kThreads - 1) / kThreads), (unsigned)((batch + chunk - 1) / chunk));
  hipLaunchKernelGGL(k_sz_counts, grid, dim3(kThreads), 0, s, M, r0, c0, w, nw, N * M, batch,
                     chunk, cfg, flags, reinterpret_cast<unsigned long long*>(same),
                     reinterpret_cast<unsigned long long*>(nsamples));
  return hipGetLastError();
}

hipError_t launch_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples,
                                   const double* trans, const int64_t* ntrans, double kx,
                                   double ky, double factor, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_structure_factor, dim3(1), dim3(kThreads), 0, s, h, w,
                     reinterpret_cast<const unsigned long long*>(same),
                     reinterpret_cast<const unsigned long long*>(nsamples), trans, ntrans, kx, ky,
                     factor, out);
  return hipGetLastError();
}

// out[0] = OR of f[0..n) (one workgroup)
__global__ void __launch_bounds__(kThreads) k_flags_or(const uint32_t* f, int n, uint32_t* out) {
  __shared__ uint32_t part[kThreads];
  uint32_t v = 0u;
  for (int e = threadIdx.x; e < n; e += blockDim.x) v |= f[e];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] |= part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

hipError_t launch_flags_or(const uint32_t* f, int n, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_flags_or, dim3(1), dim3(kThreads), 0, s, f, n, out);
  return hipGetLastError();
}

hipError_t launch_corr_init(const Lat& V, const FlipShape& z, int nv, const uint8_t* cfg_real,
                            uint8_t* cfg_inst, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_corr_init, dim3(nv), dim3(kThreads), 0, s, V, z, cfg_real, cfg_inst);
  return hipGetLastError();
}

hipError_t launch_corr_copy(const Lat& V, const Lat& R, int nbr, int v0, int count, int src_slot,
                            int dst_slot, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_corr_copy, dim3(count), dim3(kThreads), 0, s, V, R, nbr, v0, src_slot,
                     dst_slot);
  return hipGetLastError();
}

template <uint32_t GM>
static hipError_t launch_flip_row_g(const Lat& V, const Lat& R, const FlipShape& z,
                                    const BufPlan& p, int lds, int nv, hipStream_t s) {
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_flip_row<GM>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_flip_row<GM>, dim3(nv), dim3(kThreads), lds, s, V, R, z, p);
  return hipGetLastError();
}

hipError_t launch_flip_row(const Lat& V, const Lat& R, const FlipShape& z, const BufPlan& p,
                           int lds, int nv, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  if (p.glob == kSandQ) return launch_flip_row_g<kSandQ>(V, R, z, p, lds, nv, s);
  if (p.glob == kSandT2E2Q) return launch_flip_row_g<kSandT2E2Q>(V, R, z, p, lds, nv, s);
  return launch_flip_row_g<kGlobAny>(V, R, z, p, lds, nv, s);
}

hipError_t launch_corr_finish(const Lat& V, const Lat& R, const FlipShape& z, uint32_t* flags,
                              double* ratios, double* sums, int64_t* count, hipStream_t s) {
  if (z.nbr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_corr_finish, dim3(z.nbr), dim3(kThreads), 0, s, V, R, z, flags, ratios);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = z.h * z.w;
  hipLaunchKernelGGL(k_corr_sums, dim3((n * n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, V,
                     R, z, flags, sums, count);
  return hipGetLastError();
}

hipError_t launch_go_update(int64_t nparams, double* T, const double* sd, const double* sde,
                            const double* stats, double dt, const double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_go_update, dim3((unsigned)((nparams + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, nparams, T, sd, sde, stats, dt, p);
  return hipGetLastError();
}

hipError_t launch_metropolis(const Lat& L, int nb, const double* uniforms, uint8_t* cfg,
                             uint8_t* accepted, hipStream_t s) {
  hipLaunchKernelGGL(k_metropolis, dim3((nb + kThreads - 1) / kThreads), dim3(kThreads), 0, s, L,
                     nb, uniforms, cfg, accepted);
  return hipGetLastError();
}

hipError_t launch_finalize(const Lat& L, int nb, int want_eloc, double* logabs, int8_t* sign,
                           double* eloc, uint32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(kThreads), 0, s, L, want_eloc, logabs, sign, eloc,
                     flags);
  return hipGetLastError();
}

}  // namespace pg
