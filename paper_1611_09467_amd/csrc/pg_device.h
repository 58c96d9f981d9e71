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

// k-steps per group of back-to-back MFMAs in the matrix-core GEMMs
constexpr int kMfmaGroup = 2;
// largest block of reflectors applied at once in compact-WY form
constexpr int kMaxWyBlock = 16;

// rot: tile t goes to wave (t + rot) % (waves), so back-to-back calls
// without a barrier between them spread their tiles over all waves.
__device__ inline void mgemm64(int Md, int Nd, int K, const double* A, int sam, int sak,
                               const double* B, int sbk, int sbn, double* C, Map cm, Map cn,
                               double alpha, int tid, int nt, int rot = 0) {
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int tm = (Md + 15) >> 4, tn = (Nd + 15) >> 4;
  const bool unit = alpha == 1.0;
  const int li = lane & 15, lk = lane >> 4;
  // this wave's tiles t = t0, t0 + nw, ... as (row, column) = (t / tn, t % tn),
  // stepped on the scalar unit without a division
  int trow = 0, tcol = (__builtin_amdgcn_readfirstlane(wave) + nw - rot % nw) % nw;
  for (; tcol >= tn; tcol -= tn) ++trow;
  for (; trow < tm;) {
    const int m0 = trow << 4, n0 = tcol << 4;
    const int m = m0 + li, n = n0 + li;
    const bool mv = m < Md, nv = n < Nd;
    // rows / columns past the matrix read row / column 0 instead: they only
    // feed outputs that are never stored
    const double* Ap = A + (mv ? m : 0) * sam + lk * sak;
    const double* Bp = B + (nv ? n : 0) * sbn + lk * sbk;
    const int da = 4 * sak, db = 4 * sbk, nk = K >> 2;
    pg_d4 acc = {0.0, 0.0, 0.0, 0.0};
    // full k-steps in groups of kMfmaGroup, two register sets in turn: one
    // group's operands load while the other's MFMAs issue back to back.  The
    // loads are unconditional (a step past the last one rereads the last one
    // and its value goes unused), so the waits count exactly the loads in
    // flight.
    const int kl = nk > 0 ? nk - 1 : 0;
    double a0[kMfmaGroup], b0[kMfmaGroup], a1[kMfmaGroup], b1[kMfmaGroup];
    auto load = [&](int g, double* a, double* b) {
#pragma unroll
      for (int s = 0; s < kMfmaGroup; ++s) {
        const int q = g + s < kl ? g + s : kl;
        a[s] = Ap[q * da];
        b[s] = Bp[q * db];
      }
    };
    auto run = [&](int g, const double* a, const double* b) {
#pragma unroll
      for (int s = 0; s < kMfmaGroup; ++s)
        if (g + s < nk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
    };
    if (nk > 0) load(0, a0, b0);
    for (int g = 0; g < nk; g += 2 * kMfmaGroup) {
      load(g + kMfmaGroup, a1, b1);
      run(g, a0, b0);
      if (g + kMfmaGroup >= nk) break;
      load(g + 2 * kMfmaGroup, a0, b0);
      run(g + kMfmaGroup, a1, b1);
    }
    if (4 * nk < K) {  // partial last step: k past K contributes zero
      double a = 0.0, b = 0.0;
      if (4 * nk + lk < K) {
        a = Ap[nk * da];
        b = Bp[nk * db];
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
        if (mr < Md)
          C[same ? base + 4 * i * cm.s0 : mapoff(cm, mr) + cno] = unit ? acc[i] : alpha * acc[i];
      }
    }
    for (tcol += nw; tcol >= tn; tcol -= tn) ++trow;
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
  const bool unit = alpha == 1.0f;
  const int li = lane & 15, lk = lane >> 4;
  // this wave's tiles t = t0, t0 + nw, ... as (row, column) = (t / tn, t % tn),
  // stepped on the scalar unit without a division
  int trow = 0, tcol = (__builtin_amdgcn_readfirstlane(wave) + nw - rot % nw) % nw;
  for (; tcol >= tn; tcol -= tn) ++trow;
  for (; trow < tm;) {
    const int m0 = trow << 4, n0 = tcol << 4;
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
        if (mr < Md)
          C[same ? base + i * cm.s0 : mapoff(cm, mr) + cno] = (TC)(unit ? acc[i] : alpha * acc[i]);
      }
    }
    for (tcol += nw; tcol >= tn; tcol -= tn) ++trow;
  }
}

// ---------------------------------------------------------------------------
// reductions: lanes of a wave64 by butterfly shuffles, waves through LDS
// (red: at least nt/64 + 1 doubles); every thread receives the result.
// ---------------------------------------------------------------------------

// A lane permutation within each row of 16 lanes (a DPP move, no trip
// through LDS), applied to both halves of a double: CTRL 0xB1 exchanges
// lanes l and l ^ 1, 0x4E lanes l and l ^ 2, 0x141 mirrors each half row
// (l <-> 7 - l), 0x140 each row (l <-> 15 - l), 0x128 rotates each row by 8
// (l <-> l ^ 8).  Every lane of the wave must be active.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The value of lane l (uniform l).
__device__ inline double lane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// v + (v of lane l ^ 16) and v + (v of lane l ^ 32), the same in both lanes
// of each pair: the rows of 16 lanes (halves of 32) exchanged by gfx950's
// permlane swaps, both halves of the double.
__device__ inline double xsum16(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned bl = (unsigned)b, bh = (unsigned)(b >> 32);
  const auto lo = __builtin_amdgcn_permlane16_swap(bl, bl, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(bh, bh, false, false);
  const double x = __longlong_as_double(((long long)hi[0] << 32) | (long long)lo[0]);
  const double y = __longlong_as_double(((long long)hi[1] << 32) | (long long)lo[1]);
  return x + y;
}

__device__ inline double xsum32(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned bl = (unsigned)b, bh = (unsigned)(b >> 32);
  const auto lo = __builtin_amdgcn_permlane32_swap(bl, bl, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(bh, bh, false, false);
  const double x = __longlong_as_double(((long long)hi[0] << 32) | (long long)lo[0]);
  const double y = __longlong_as_double(((long long)hi[1] << 32) | (long long)lo[1]);
  return x + y;
}

// Sum over each group of 8 lanes (l / 8 fixed), the same value in all 8:
// pairs, quads, then the two quads of a half row.
__device__ inline double sum8(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  return v + dpp_f64<0x141>(v);
}

// Butterfly sums and maxima over the 64 lanes, identical in every lane: the
// steps inside a row of 16 lanes by DPP, then the four row results read
// back as uniform values.
__device__ inline double wave_sum(double v) {
  v = sum8(v);
  v += dpp_f64<0x140>(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
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

// The same LQ for one wave with W held in registers: lane l holds columns l
// and l + 64 of rows 0 .. RM-1 (r <= RM, c <= 128), so the dot products of a
// reflector with every remaining row reduce together, without memory round
// trips.  W is read (global or LDS); the reflectors go to vbuf (k x c, LDS)
// and tau (k, LDS), L (r x k) and Q (k x c) are written as by lq_householder.
template <int RM>
__device__ inline void lq_wave(const double* W, int r, int c, double* Q, double* L, double* vbuf,
                               double* tau, int lane) {
  const int k = r < c ? r : c;
  const int t0 = lane, t1 = lane + 64;
  const bool h0 = t0 < c, h1 = t1 < c;
  double w0[RM], w1[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    w0[j] = (j < r && h0) ? W[j * c + t0] : 0.0;
    w1[j] = (j < r && h1) ? W[j * c + t1] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    if (i < k) {  // constant trip count, predicated body: the arrays stay in registers
    const double part = (t0 > i ? w0[i] * w0[i] : 0.0) + w1[i] * w1[i];
    const double sigma = wave_sum(part);
    const double alpha = lane_f64(w0[i], i);  // W[i][i] (i < 64), a uniform value
    double ti = 0.0, beta = alpha, scale = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      ti = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    const double v0 = t0 < i ? 0.0 : (t0 == i ? 1.0 : w0[i] * scale);
    const double v1 = w1[i] * scale;  // columns >= 64 > i
    if (h0) vbuf[i * c + t0] = v0;
    if (h1) vbuf[i * c + t1] = v1;
    if (lane == 0) tau[i] = ti;
    if (ti != 0.0) {
      double d[RM];
#pragma unroll
      for (int j = 0; j < RM; ++j) d[j] = (j > i && j < r) ? fma(w0[j], v0, w1[j] * v1) : 0.0;
#pragma unroll
      for (int j = 0; j < RM; ++j)
        if (j > i) d[j] = wave_sum(d[j]);
#pragma unroll
      for (int j = 0; j < RM; ++j)
        if (j > i) {
          const double f = ti * d[j];
          w0[j] = fma(-f, v0, w0[j]);
          w1[j] = fma(-f, v1, w1[j]);
        }
    }
    // row i: beta on the diagonal, zero to its right; L entries left of it stay
    if (t0 == i) w0[i] = beta;
    else if (t0 > i) w0[i] = 0.0;
    w1[i] = 0.0;
    }
  }
  if (t0 < k) {
#pragma unroll
    for (int j = 0; j < RM; ++j)
      if (j < r) L[j * k + t0] = t0 <= j ? w0[j] : 0.0;
  }
  // Q = [I_k 0] H_{k-1} ... H_0, rows of Q in the same lane layout
  double q0[RM], q1[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) {
    q0[a] = t0 == a ? 1.0 : 0.0;
    q1[a] = 0.0;
  }
  wave_sync();
#pragma unroll
  for (int i = RM - 1; i >= 0; --i) {
    const double ti = i < k ? tau[i] : 0.0;
    if (ti != 0.0) {
    const double v0 = h0 ? vbuf[i * c + t0] : 0.0, v1 = h1 ? vbuf[i * c + t1] : 0.0;
    double d[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) d[a] = a < k ? fma(q0[a], v0, q1[a] * v1) : 0.0;
#pragma unroll
    for (int a = 0; a < RM; ++a) d[a] = wave_sum(d[a]);
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      const double f = ti * d[a];
      q0[a] = fma(-f, v0, q0[a]);
      q1[a] = fma(-f, v1, q1[a]);
    }
    }
  }
#pragma unroll
  for (int a = 0; a < RM; ++a) {
    if (a < k && h0) Q[a * c + t0] = q0[a];
    if (a < k && h1) Q[a * c + t1] = q1[a];
  }
  wave_sync();
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

// One step of Gaussian elimination with partial pivoting on T - lam I (T
// tridiagonal with zero diagonal, gn = -lam), fused with the forward
// substitution.  State: gi (the pivot candidate of row i), ui (its
// superdiagonal), xi (its right-hand side); inputs: li = e[i] (the
// subdiagonal below it), un = e[i+1] (0 past the end) and xn (the next
// right-hand side entry).  Outputs: U row i as its reciprocal pivot rp (a
// pivot below tiny is replaced by tiny) and superdiagonals du, du2, and the
// eliminated right-hand side xr; the state moves to row i + 1.
__device__ __forceinline__ void ge_step(double li, double un, double xn, double gn, double tiny,
                                        double& gi, double& ui, double& xi, double& rp,
                                        double& du, double& du2, double& xr) {
  const bool sw = fabs(gi) < fabs(li);  // row interchange when the subdiagonal entry is the larger
  const double piv = sw ? li : gi, oth = sw ? gi : li;
  const double pg = fabs(piv) < tiny ? (piv < 0.0 ? -tiny : tiny) : piv;
  rp = recip_nr(pg);
  const double f = oth * rp;
  du = sw ? gn : ui;
  du2 = sw ? un : 0.0;
  xr = sw ? xn : xi;
  const double xnew = sw ? xi - f * xn : xn - f * xi;
  const double gnew = sw ? ui - f * gn : gn - f * ui;
  ui = sw ? -f * un : un;
  xi = xnew;
  gi = gnew;
}

// Entry i of the fixed start vector of inverse iteration (in [1, 1.5)).
__device__ inline double ii_start(int i, int seed) {
  const double h = (double)((i * 7919 + seed * 104729 + 17) % 1009) * (1.0 / 1009.0);
  return 1.0 + 0.5 * h;
}

// Inverse iteration for one eigenvalue lam of a symmetric tridiagonal with
// zero diagonal (the Golub-Kahan form) and off-diagonal e[0..n-2]: `iters`
// solves of (T - lam I) y = x, the first from a fixed start vector, each
// later one from the previous solution scaled to unit maximum, each by the
// elimination of ge_step and back substitution.  The elimination is a
// sequential recurrence carried in registers.  Its factors are not stored:
// the forward sweep keeps its state at the start of every chunk of kIiChunk
// steps (a checkpoint), and the back substitution recomputes each chunk's
// factors from its checkpoint into registers, last chunk first.  That doubles
// the elimination arithmetic but leaves one vector read and one written per
// solve; the next chunk's operands are loaded while the current one runs.
// Vectors and checkpoints are strided by ss, so that the vectors of a batch,
// computed on adjacent lanes, are interleaved in memory.  On return x[0..n)
// holds the last solution and *scale the factor that brings it to unit
// 2-norm (applied as (x / max |x|) / norm); w: a second vector (n) and
// 3 ceil((n - 1) / kIiChunk) checkpoint entries.
constexpr int kIiChunk = 4;

__device__ __forceinline__ void tgk_inverse_iteration(const double* __restrict__ e, int n,
                                                      double lam, double tiny, int seed, int iters,
                                                      double* __restrict__ x,
                                                      double* __restrict__ w, double* scale_max,
                                                      double* scale_norm, int ss) {
  constexpr int C = kIiChunk;
  const int nsteps = n - 1;  // elimination steps 0 .. n-2
  const int nck = (nsteps + C - 1) / C;
  double* __restrict__ y = w;
  double* __restrict__ ck = w + (int64_t)n * ss;  // checkpoint q of chunk c at (3 c + q) ss
  const double gn = -lam;
  const double* src = nullptr;  // the previous solution (none in the first solve)
  double sc = 1.0;              // 1 / its largest magnitude
  // right-hand side entries i0 .. i0 + C - 1 (0 past the end)
  auto rhs = [&](int i0, double* v) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int i = i0 + u;
      v[u] = i < n ? (src ? src[(int64_t)i * ss] * sc : ii_start(i, seed)) : 0.0;
    }
  };
  double* dst = x;
  for (int it = 0; it < iters; ++it) {
    dst = ((iters - 1 - it) & 1) ? y : x;  // the last solve lands in x
    // ---- forward sweep: checkpoints only
    double gi = gn, ui = n > 1 ? e[0] : 0.0;
    double xi = src ? src[0] * sc : ii_start(0, seed);
    double nb[C];
    rhs(1, nb);
    for (int c = 0; c < nck; ++c) {
      double cur[C];
#pragma unroll
      for (int u = 0; u < C; ++u) cur[u] = nb[u];
      rhs((c + 1) * C + 1, nb);
      ck[(int64_t)(3 * c) * ss] = gi;
      ck[(int64_t)(3 * c + 1) * ss] = ui;
      ck[(int64_t)(3 * c + 2) * ss] = xi;
#pragma unroll
      for (int u = 0; u < C; ++u) {
        const int i = c * C + u;
        if (i < nsteps) {
          double rp, du, du2, xr;
          ge_step(e[i], i + 2 < n ? e[i + 1] : 0.0, cur[u], gn, tiny, gi, ui, xi, rp, du, du2, xr);
        }
      }
    }
    // ---- back substitution, chunk by chunk from the end
    const double gl = fabs(gi) < tiny ? (gi < 0.0 ? -tiny : tiny) : gi;
    double a1 = xi * recip_nr(gl), a2 = 0.0;
    dst[(int64_t)(n - 1) * ss] = a1;
    double m = fabs(a1);
    double pk[3] = {0.0, 0.0, 0.0};
    if (nck > 0) {
      const int c = nck - 1;
      pk[0] = ck[(int64_t)(3 * c) * ss];
      pk[1] = ck[(int64_t)(3 * c + 1) * ss];
      pk[2] = ck[(int64_t)(3 * c + 2) * ss];
      rhs(c * C + 1, nb);
    }
    for (int c = nck - 1; c >= 0; --c) {
      double g = pk[0], uu = pk[1], xv = pk[2], cur[C];
#pragma unroll
      for (int u = 0; u < C; ++u) cur[u] = nb[u];
      if (c > 0) {
        pk[0] = ck[(int64_t)(3 * c - 3) * ss];
        pk[1] = ck[(int64_t)(3 * c - 2) * ss];
        pk[2] = ck[(int64_t)(3 * c - 1) * ss];
        rhs((c - 1) * C + 1, nb);
      }
      double R[C], DU[C], DU2[C], XR[C];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        const int i = c * C + u;
        R[u] = DU[u] = DU2[u] = XR[u] = 0.0;
        if (i < nsteps)
          ge_step(e[i], i + 2 < n ? e[i + 1] : 0.0, cur[u], gn, tiny, g, uu, xv, R[u], DU[u], DU2[u],
                  XR[u]);
      }
#pragma unroll
      for (int u = C - 1; u >= 0; --u) {
        const int i = c * C + u;
        if (i < nsteps) {
          // the last row has no second superdiagonal term (a2 = 0 there)
          const double v = (XR[u] - DU[u] * a1 - DU2[u] * a2) * R[u];
          dst[(int64_t)i * ss] = v;
          a2 = a1;
          a1 = v;
          m = fmax(m, fabs(v));
        }
      }
    }
    sc = m > 0.0 ? 1.0 / m : 0.0;
    src = dst;
  }
  double sq = 0.0;
  for (int i0 = 0; i0 < n; i0 += C) {
    double t[C];
    rhs(i0, t);  // x scaled to unit maximum
#pragma unroll
    for (int u = 0; u < C; ++u) sq += t[u] * t[u];
  }
  *scale_max = sc;
  *scale_norm = sq > 0.0 ? 1.0 / sqrt(sq) : 0.0;
}

// Sturm counts: the number of eigenvalues below each of P points x[0..P)
// of the symmetric tridiagonal with zero diagonal and squared off-diagonal
// e2, as the number of sign changes of the leading principal minors
// p_i(x) = -x p_{i-1} - e2_{i-1} p_{i-2} (p_{-1} = 0, p_0 = 1): no division.
// The caller scales the matrix by a power of two to norm <= 1, so |p_i|
// grows at most threefold per step and a check every 8 steps, rescaling the
// pair (p_{i-1}, p_i) by an exact power of two when its larger member leaves
// [2^-500, 2^500], keeps it in range.  A minor that vanishes exactly counts
// as a sign change (the limit from below the eigenvalue of the leading
// block).  The P recurrences are interleaved.
template <int P>
__device__ inline void sturm_count(const double* __restrict__ e2, int n, const double* x, int* c) {
  double p0[P], p1[P];
  int cc[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    p0[q] = 1.0;
    p1[q] = -x[q];
    if (p1[q] == 0.0) p1[q] = -0x1p-600;
    cc[q] = p1[q] < 0.0;
  }
  auto step = [&](double ei) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      double pn = -x[q] * p1[q] - ei * p0[q];
      if (pn == 0.0) pn = p1[q] < 0.0 ? 0x1p-600 : -0x1p-600;
      cc[q] += (pn < 0.0) != (p1[q] < 0.0);
      p0[q] = p1[q];
      p1[q] = pn;
    }
  };
  int i = 1;
  // blocks of 8 steps: the block's e^2 are loaded together, then the range check
  for (; i + 8 <= n; i += 8) {
    double eb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) eb[u] = e2[i + u - 1];
#pragma unroll
    for (int u = 0; u < 8; ++u) step(eb[u]);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const double a = fmax(fabs(p0[q]), fabs(p1[q]));
      if (a > 0x1p500 || a < 0x1p-500) {
        const int ex = ilogb(a);
        p0[q] = ldexp(p0[q], -ex);
        p1[q] = ldexp(p1[q], -ex);
      }
    }
  }
  for (; i < n; ++i) step(e2[i - 1]);
#pragma unroll
  for (int q = 0; q < P; ++q) c[q] = cc[q];
}

// Householder tridiagonalisation with the matrix held in registers: the 256
// threads form a 16 x 16 grid, thread (tr, tc) = (tid / 16, tid % 16) holding
// rows tr + 16 x and columns tc + 16 y (x, y < NB, n <= 16 NB), so the active
// part stays spread over all threads as it shrinks.  Per reflector: the
// column is published through LDS, one wave forms the reflector, then the
// product p = tau A v (row sums across the 16 lanes of a row group) and the
// rank-2 update A -= v w^T + w v^T run on the registers.  Output: d, e, tau,
// and reflector i (entries i+1 .. n-1, the first being 1) contiguous in row i

// ---------------------------------------------------------------------------
// Leading singular triplets of a dense matrix X (rows x cols, row-major,
// ld = cols), backward stable in X:
//   1. Householder bidiagonalisation A = Q_L [B; 0] Q_R^T of the tall
//      orientation A = X (rows >= cols) or A = X^T, B upper bidiagonal;
//   2. the largest singular values by bisection on Sturm counts of the
//      Golub-Kahan tridiagonal T_GK of B (zero diagonal, off-diagonal
//      B00, B01, B11, B12, ...), whose eigenvalues are +-sigma;
//   3. eigenvectors of T_GK by inverse iteration: their odd entries are the
//      left, their even entries the right singular vectors of B;
//   4. orthonormalisation; 5. back-transformation by the stored reflectors
//      (Q_L when X is tall, Q_R of X^T when X is wide).
// This is the bidiagonal-SVD route of LAPACK's dbdsvdx (bisection and
// inverse iteration on the Golub-Kahan tridiagonal).  X is never squared, so
// the kept subspace errs by O(eps ||X|| / (sigma_k - sigma_{k+1})), as for
// any backward-stable SVD.
//
// On exit sv[0..kk) holds the kk = min(k+1, min(rows, cols)) largest singular
// values in decreasing order, and U the k leading left singular vectors,
// vector t at U[t*rows .. t*rows + rows).  X is not modified.
// W: rows*cols doubles (the matrix being reduced, then the stored
// reflectors); wk: top_svd_work(rows, cols, k, nt == 64) doubles (a one-wave
// workgroup needs rows, cols <= 72); lw: lwn doubles of
// per-vector inverse-iteration scratch (8 min(rows, cols) doubles per vector,
// kb vectors at a time), reused for the orthonormalisation, the compact-WY
// back-transformation and the Sturm counts (lwn >= 2 nt); sm: smn doubles of
// fast (LDS) scratch that, where large enough, holds the small matrices of
// the orthonormalisation and of the back-transformation instead of lw.
// ---------------------------------------------------------------------------
__host__ __device__ inline int top_svd_work(int rows, int cols, int k, int one_wave) {
  const int m = rows > cols ? rows : cols, n = rows < cols ? rows : cols;
  const int compact = 6 * n + m + 64 + 4 * (k + 2) + 16;  // the one-wave register path
  return one_wave ? compact : compact + 2 * m + 5 * n;      // + in-memory / four-wave arrays
}

// Householder vector of x[0..len) (x[0] = alpha, s = sum of the others'
// squares): (I - tau v v^T) x = beta e_0 with v[0] = 1, v[i] = x[i] * scale.
__device__ inline void house_coeffs(double alpha, double s, double* tau, double* beta,
                                    double* scale) {
  *tau = 0.0;
  *beta = alpha;
  *scale = 0.0;
  if (s > 0.0) {
    const double nrm = sqrt(alpha * alpha + s);
    *beta = alpha >= 0.0 ? -nrm : nrm;
    *tau = (*beta - alpha) / *beta;
    *scale = 1.0 / (alpha - *beta);
  }
}

// Bidiagonalisation with A in registers (m <= 16 NB <= 128, 256 threads): thread
// (tr, tc) = (tid / 16, tid % 16) holds rows tr + 16 x and columns tc + 16 y
// (x, y < NB).  Step i publishes column i through LDS; every wave forms the
// left reflector from it by itself (no barrier); the column sums v^T A are
// combined over the four waves through LDS (one barrier).  Row i is then
// published (one barrier), every wave forms the right reflector, and the row
// sums A v stay inside 16-lane groups (shuffles only).  B goes to
// t[2i] = B[i][i], t[2i+1] = B[i][i+1]; the reflectors of Q_L (keep_left) or
// of Q_R go to rows of R (reflector i at R[i*ldr], starting with its leading
// 1), their factors to tq.
template <int NB>
__device__ inline void bidiag_reg(const double* X, int ldx, int trans, int m, int n,
                                  int keep_left, double* t, double* tq, double* R, int ldr,
                                  double* colbuf, double* rowbuf, double* part, int tid) {
  const int tr = tid >> 4, tc = tid & 15, lane = tid & 63, wave = tid >> 6;
  double a[NB][NB];
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int r = tr + 16 * x, c = tc + 16 * y;
      a[x][y] = (r < m && c < n) ? (trans ? X[c * ldx + r] : X[r * ldx + c]) : 0.0;
    }
  for (int i = 0; i < n; ++i) {
    const int ib = i >> 4, ic = i & 15;
    // (1) column i, rows i .. m-1
    if (tc == ic) {
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const int r = tr + 16 * x;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y) v = y == ib ? a[x][y] : v;
        if (r >= i && r < m) colbuf[r] = v;
      }
    }
    __syncthreads();
    // (2) left reflector (identical in every wave: same data, same reduction order)
    double s = 0.0;
    for (int r = i + 1 + lane; r < m; r += 64) s += colbuf[r] * colbuf[r];
    s = wave_sum(s);
    double tl, beta, scale;
    house_coeffs(colbuf[i], s, &tl, &beta, &scale);
    if (keep_left && wave == 0) {
      for (int r = i + lane; r < m; r += 64) R[i * ldr + (r - i)] = r == i ? 1.0 : colbuf[r] * scale;
      if (lane == 0) tq[i] = tl;
    }
    if (tid == 0) t[2 * i] = beta;
    // (3) A -= v (tl v^T A) on the columns right of i
    if (tl != 0.0) {
      double vr[NB];
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const int r = tr + 16 * x;
        vr[x] = (r < i || r >= m) ? 0.0 : (r == i ? 1.0 : colbuf[r] * scale);
      }
      double ps[NB];
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        double q = 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x) q = fma(vr[x], a[x][y], q);
        q = xsum32(xsum16(q));  // over the four rows of 16 lanes (tr) of the wave
        ps[y] = q;
      }
      if (lane < 16) {
#pragma unroll
        for (int y = 0; y < NB; ++y) {
          const int c = tc + 16 * y;
          if (c < n) part[wave * n + c] = ps[y];
        }
      }
      __syncthreads();
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const int c = tc + 16 * y;
        const double w =
            (c > i && c < n) ? tl * ((part[c] + part[n + c]) + (part[2 * n + c] + part[3 * n + c]))
                             : 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x) a[x][y] = fma(-vr[x], w, a[x][y]);
      }
    }
    if (i + 1 >= n) break;
    // (4) row i, columns i+1 .. n-1
    if (tr == ic) {
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const int c = tc + 16 * y;
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x) v = x == ib ? a[x][y] : v;
        if (c > i && c < n) rowbuf[c] = v;
      }
    }
    __syncthreads();
    if (i + 2 >= n) {
      if (tid == 0) t[2 * i + 1] = rowbuf[i + 1];
      continue;
    }
    // (5) right reflector on columns i+1 .. n-1 (every wave)
    double s2 = 0.0;
    for (int c = i + 2 + lane; c < n; c += 64) s2 += rowbuf[c] * rowbuf[c];
    s2 = wave_sum(s2);
    double tg, b2, sc2;
    house_coeffs(rowbuf[i + 1], s2, &tg, &b2, &sc2);
    if (!keep_left && wave == 0) {
      for (int c = i + 1 + lane; c < n; c += 64)
        R[i * ldr + (c - i - 1)] = c == i + 1 ? 1.0 : rowbuf[c] * sc2;
      if (lane == 0) tq[i] = tg;
    }
    if (tid == 0) t[2 * i + 1] = b2;
    // (6) A -= (tg A v) v^T on the rows below i
    if (tg != 0.0) {
      double vc[NB];
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const int c = tc + 16 * y;
        vc[y] = (c <= i || c >= n) ? 0.0 : (c == i + 1 ? 1.0 : rowbuf[c] * sc2);
      }
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        double q = 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y) q = fma(a[x][y], vc[y], q);
        q = sum8(q);  // over the 16 lanes of a row (tc)
        q += dpp_f64<0x140>(q);
        const int r = tr + 16 * x;
        const double w = (r > i && r < m) ? tg * q : 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y) a[x][y] = fma(-w, vc[y], a[x][y]);
      }
    }
  }
  __syncthreads();
}

// The same for a workgroup of one wave (64 threads): lane (tr, tc) =
// (lane / 8, lane % 8) holds rows tr + 8 x and columns tc + 8 y (x, y < NB,
// m <= 8 NB).  Column sums (over tr) and row sums (over tc) are lane
// shuffles; only the published column and row go through LDS.  Blocks of
// rows or columns that lie wholly before the active corner are skipped
// (a condition that is the same on every lane).
template <int NB>
__device__ inline void bidiag_wave(const double* X, int ldx, int trans, int m, int n,
                                   int keep_left, double* t, double* tq, double* R, int ldr,
                                   double* colbuf, double* rowbuf, int lane) {
  const int tr = lane >> 3, tc = lane & 7;
  double a[NB][NB];
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int r = tr + 8 * x, c = tc + 8 * y;
      a[x][y] = (r < m && c < n) ? (trans ? X[c * ldx + r] : X[r * ldx + c]) : 0.0;
    }
  for (int i = 0; i < n; ++i) {
    const int ib = i >> 3, ic = i & 7;
    // (1) column i, rows i .. m-1
    if (tc == ic) {
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        if (8 * x + 7 < i) continue;
        const int r = tr + 8 * x;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y) v = y == ib ? a[x][y] : v;
        if (r >= i && r < m) colbuf[r] = v;
      }
    }
    __syncthreads();
    // (2) left reflector
    double s = 0.0;
    for (int r = i + 1 + lane; r < m; r += 64) s += colbuf[r] * colbuf[r];
    s = wave_sum(s);
    double tl, beta, scale;
    house_coeffs(colbuf[i], s, &tl, &beta, &scale);
    if (keep_left) {
      for (int r = i + lane; r < m; r += 64) R[i * ldr + (r - i)] = r == i ? 1.0 : colbuf[r] * scale;
      if (lane == 0) tq[i] = tl;
    }
    if (lane == 0) t[2 * i] = beta;
    // (3) A -= v (tl v^T A) on the columns right of i
    if (tl != 0.0) {
      double vr[NB];
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const int r = tr + 8 * x;
        vr[x] = (r < i || r >= m) ? 0.0 : (r == i ? 1.0 : colbuf[r] * scale);
      }
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        if (8 * y + 7 <= i) continue;
        double q = 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x)
          if (8 * x + 7 >= i) q = fma(vr[x], a[x][y], q);
        q += dpp_f64<0x128>(q);  // lane ^ 8
        q = xsum32(xsum16(q));
        const int c = tc + 8 * y;
        const double w = (c > i && c < n) ? tl * q : 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x)
          if (8 * x + 7 >= i) a[x][y] = fma(-vr[x], w, a[x][y]);
      }
    }
    if (i + 1 >= n) break;
    // (4) row i, columns i+1 .. n-1
    if (tr == ic) {
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        if (8 * y + 7 <= i) continue;
        const int c = tc + 8 * y;
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x) v = x == ib ? a[x][y] : v;
        if (c > i && c < n) rowbuf[c] = v;
      }
    }
    __syncthreads();
    if (i + 2 >= n) {
      if (lane == 0) t[2 * i + 1] = rowbuf[i + 1];
      continue;
    }
    // (5) right reflector on columns i+1 .. n-1
    double s2 = 0.0;
    for (int c = i + 2 + lane; c < n; c += 64) s2 += rowbuf[c] * rowbuf[c];
    s2 = wave_sum(s2);
    double tg, b2, sc2;
    house_coeffs(rowbuf[i + 1], s2, &tg, &b2, &sc2);
    if (!keep_left) {
      for (int c = i + 1 + lane; c < n; c += 64)
        R[i * ldr + (c - i - 1)] = c == i + 1 ? 1.0 : rowbuf[c] * sc2;
      if (lane == 0) tq[i] = tg;
    }
    if (lane == 0) t[2 * i + 1] = b2;
    // (6) A -= (tg A v) v^T on the rows below i
    if (tg != 0.0) {
      double vc[NB];
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const int c = tc + 8 * y;
        vc[y] = (c <= i || c >= n) ? 0.0 : (c == i + 1 ? 1.0 : rowbuf[c] * sc2);
      }
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        if (8 * x + 7 <= i) continue;
        double q = 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y)
          if (8 * y + 7 > i) q = fma(a[x][y], vc[y], q);
        q = sum8(q);
        const int r = tr + 8 * x;
        const double w = (r > i && r < m) ? tg * q : 0.0;
#pragma unroll
        for (int y = 0; y < NB; ++y)
          if (8 * y + 7 > i) a[x][y] = fma(-w, vc[y], a[x][y]);
      }
    }
  }
  __syncthreads();
}

// The same with A (m x n, row-major) in memory (LDS or global), any m.  The
// reflectors are kept in place: left reflector i in column i from row i down
// (keep_left), right reflector i in row i from column i+1 on, each with its
// leading 1 stored.  vb: m, vb2: n, wv: n, pv: m, red: 2.
__device__ inline void bidiag_loop(double* W, int m, int n, int keep_left, double* t, double* tq,
                                   double* vb, double* vb2, double* wv, double* pv, double* red,
                                   int tid, int nt) {
  const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
  for (int i = 0; i < n; ++i) {
    if (wave == 0) {
      double s = 0.0;
      for (int r = i + 1 + lane; r < m; r += 64) s += W[r * n + i] * W[r * n + i];
      s = wave_sum(s);
      double tl, beta, scale;
      house_coeffs(W[i * n + i], s, &tl, &beta, &scale);
      for (int r = i + lane; r < m; r += 64) {
        const double v = r == i ? 1.0 : W[r * n + i] * scale;
        vb[r] = v;
        if (keep_left) W[r * n + i] = v;
      }
      if (lane == 0) {
        t[2 * i] = beta;
        red[0] = tl;
        if (keep_left) tq[i] = tl;
      }
    }
    __syncthreads();
    const double tl = red[0];
    const int nc = n - i - 1;
    if (tl != 0.0 && nc > 0) {
      for (int c = i + 1 + tid; c < n; c += nt) {
        double q = 0.0;
        for (int r = i; r < m; ++r) q = fma(vb[r], W[r * n + c], q);
        wv[c] = tl * q;
      }
      __syncthreads();
      for (int e = tid; e < (m - i) * nc; e += nt) {
        const int r = i + e / nc, c = i + 1 + e % nc;
        W[r * n + c] = fma(-vb[r], wv[c], W[r * n + c]);
      }
      __syncthreads();
    }
    if (i + 1 >= n) break;
    if (i + 2 >= n) {
      if (tid == 0) t[2 * i + 1] = W[i * n + i + 1];
      __syncthreads();
      continue;
    }
    if (wave == 0) {
      double s = 0.0;
      for (int c = i + 2 + lane; c < n; c += 64) s += W[i * n + c] * W[i * n + c];
      s = wave_sum(s);
      double tg, b2, sc2;
      house_coeffs(W[i * n + i + 1], s, &tg, &b2, &sc2);
      wave_sync();
      for (int c = i + 1 + lane; c < n; c += 64) {
        const double v = c == i + 1 ? 1.0 : W[i * n + c] * sc2;
        vb2[c] = v;
        if (!keep_left) W[i * n + c] = v;
      }
      if (lane == 0) {
        t[2 * i + 1] = b2;
        red[1] = tg;
        if (!keep_left) tq[i] = tg;
      }
    }
    __syncthreads();
    const double tg = red[1];
    if (tg != 0.0) {
      for (int r = i + 1 + wave; r < m; r += nw) {
        double q = 0.0;
        for (int c = i + 1 + lane; c < n; c += 64) q = fma(W[r * n + c], vb2[c], q);
        q = wave_sum(q);
        if (lane == 0) pv[r] = tg * q;
      }
      __syncthreads();
      for (int e = tid; e < (m - i - 1) * nc; e += nt) {
        const int r = i + 1 + e / nc, c = i + 1 + e % nc;
        W[r * n + c] = fma(-pv[r], vb2[c], W[r * n + c]);
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

// One eigenvector of the Golub-Kahan tridiagonal (off-diagonal tt, order 2n)
// for the eigenvalue lam by inverse iteration; its odd (half = 1) or even
// (half = 0) entries go to y[0..n), zeros to y[n..len).  scr: the vector
// (2n) and the iteration's work (2n + 3 ceil((2n - 1) / kIiChunk) <= 6n),
// every entry strided by ss.
__device__ inline void tgk_vector(const double* tt, int n, double lam, double tiny, int seed,
                                  int half, double* y, int len, double* scr, int ss) {
  double* z = scr;
  double smax, snorm;
  tgk_inverse_iteration(tt, 2 * n, lam, tiny, seed, 2, z, scr + 2 * (int64_t)n * ss, &smax, &snorm,
                        ss);
  for (int i0 = 0; i0 < n; i0 += kIiChunk) {
    double t[kIiChunk];
#pragma unroll
    for (int u = 0; u < kIiChunk; ++u) t[u] = i0 + u < n ? z[(int64_t)(2 * (i0 + u) + half) * ss] : 0.0;
#pragma unroll
    for (int u = 0; u < kIiChunk; ++u)
      if (i0 + u < n) y[i0 + u] = (t[u] * smax) * snorm;
  }
  for (int i = n; i < len; ++i) y[i] = 0.0;
}

__device__ __forceinline__ void top_svd(const double* X, int rows, int cols, int k, double* sv,
                                        double* U, double* W, double* wk, double* lw, int lwn,
                                        double* sm, int smn, int kb, int tid, int nt) {
  const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
  const int tall = rows >= cols;
  const int m = tall ? rows : cols, n = tall ? cols : rows, n2 = 2 * n;
  double* tt = wk;              // the off-diagonal of T_GK (2n - 1; its diagonal is zero)
  double* e2s = tt + n2;        // squared and scaled for the Sturm counts
  double* tq = e2s + n2;        // n reflector factors
  double* colbuf = tq + n;      // m
  double* vb2 = colbuf + m;     // n
  double* red = vb2 + n;        // 64
  double* iv = red + 64;        // 4 (k + 2) interval ends
  // arrays of the in-memory and four-wave paths only
  double* vb = iv + 4 * (k + 2) + 16;  // m
  double* pv = vb + m;                 // m
  double* wv = pv + m;                 // n
  double* part = wv + n;               // 4n
  double* Y = U;                // singular vectors of B, back-transformed in place
  const int kk = k + 1 < n ? k + 1 : n;
  const int half = tall ? 1 : 0;  // the entries of the T_GK eigenvectors that hold U
  const int o = tall ? 0 : 1;     // reflector i acts on coordinates i + o .. rows - 1
  const int nref = tall ? n : (n > 2 ? n - 2 : 0);
  for (int i = tid; i < n2; i += nt) tt[i] = 0.0;
  __syncthreads();

  // ---- 1. bidiagonalisation; reflector i entry r (r = 0: the leading 1) at rp[i ri + r rs]
  const bool wreg = nt == 64 && m <= 72;
  const bool vrow = (nt == 256 && m <= 128) || wreg;
  const double* rp;
  int ri, rs;
  if (wreg) {
    switch ((m + 7) >> 3) {
      case 1: bidiag_wave<1>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 2: bidiag_wave<2>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 3: bidiag_wave<3>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 4: bidiag_wave<4>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 5: bidiag_wave<5>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 6: bidiag_wave<6>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 7: bidiag_wave<7>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      case 8: bidiag_wave<8>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
      default: bidiag_wave<9>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, lane); break;
    }
    rp = W;
    ri = rows;
    rs = 1;
  } else if (vrow) {
    switch ((m + 15) >> 4) {
      case 1: bidiag_reg<1>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 2: bidiag_reg<2>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 3: bidiag_reg<3>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 4: bidiag_reg<4>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 5: bidiag_reg<5>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 6: bidiag_reg<6>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      case 7: bidiag_reg<7>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
      default: bidiag_reg<8>(X, cols, !tall, m, n, tall, tt, tq, W, rows, colbuf, vb2, part, tid); break;
    }
    rp = W;
    ri = rows;
    rs = 1;
  } else {
    for (int e = tid; e < m * n; e += nt) {
      const int r = e / n, c = e - r * n;
      W[e] = tall ? X[r * cols + c] : X[c * cols + r];
    }
    __syncthreads();
    bidiag_loop(W, m, n, tall, tt, tq, vb, vb2, wv, pv, red, tid, nt);
    rp = tall ? W : W + 1;
    ri = n + 1;
    rs = tall ? n : 1;
  }
  __syncthreads();

  // ---- 2. the kk largest eigenvalues of T_GK (the kk largest sigma) by
  // multisection on Sturm counts
  double hi = 0.0, emax2 = 0.0;
  for (int i = 0; i + 1 < n2; ++i) {
    const double off = fabs(tt[i]) + (i + 2 < n2 ? fabs(tt[i + 1]) : 0.0);
    hi = fmax(hi, off);
    emax2 = fmax(emax2, tt[i] * tt[i]);
  }
  hi = fmax(hi, n2 > 1 ? fabs(tt[0]) : 0.0);
  const double tnorm = hi;
  const double pivmin = 1e-290 * fmax(1.0, emax2);
  const double slack = 2.3e-16 * tnorm * n2 + 2.0 * pivmin;
  const double lo = -slack;  // the kk largest eigenvalues are >= 0
  hi += slack;
  // T_GK scaled by a power of two to norm <= 1 for the division-free recurrences
  const double tsc = tnorm > 0.0 ? ldexp(1.0, -(ilogb(tnorm) + 1)) : 1.0;
  for (int i = tid; i + 1 < n2; i += nt) e2s[i] = (tt[i] * tsc) * (tt[i] * tsc);
  if (tid < kk) {
    iv[2 * tid] = lo;
    iv[2 * tid + 1] = hi;
  }
  __syncthreads();
  // Points per thread: the recurrences are issue-bound, so one point per
  // thread (more, shorter passes) when a target has four threads or more.
  const int tpt = nt / kk < 63 ? nt / kk : 63;  // threads per target
  const int ppt = tpt >= 4 ? 1 : (tpt >= 2 ? 2 : 4);
  const int per = ppt * tpt;                     // evaluation points per target and pass
  int* cnti = reinterpret_cast<int*>(lw);
  for (int it = 0; it < 64; ++it) {
    const int tg = tid / tpt, g = tid - tg * tpt;
    if (tg < kk) {
      const double a = iv[2 * tg], b = iv[2 * tg + 1];
      double xs[4];
      int cc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xs[q] = (a + (b - a) * (ppt * g + q + 1) / (per + 1)) * tsc;
      if (ppt == 1)
        sturm_count<1>(e2s, n2, xs, cc);
      else if (ppt == 2)
        sturm_count<2>(e2s, n2, xs, cc);
      else
        sturm_count<4>(e2s, n2, xs, cc);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < ppt) cnti[tg * per + ppt * g + q] = cc[q];
    }
    __syncthreads();
    double width = 0.0;
    if (tg < kk) {
      const int target = n2 - 1 - tg;
      const double a = iv[2 * tg], b = iv[2 * tg + 1];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= ppt) break;
        const int p = ppt * g + q;
        const bool le = cnti[tg * per + p] <= target;
        const bool next_gt = p + 1 == per || cnti[tg * per + p + 1] > target;
        const bool first_gt = p == 0 && !le;
        if ((le && next_gt) || first_gt) {
          const double lo2 = first_gt ? a : a + (b - a) * (p + 1) / (per + 1);
          const double hi2 = first_gt ? a + (b - a) / (per + 1)
                                      : (p + 1 == per ? b : a + (b - a) * (p + 2) / (per + 1));
          iv[2 * kk + 2 * tg] = lo2;
          iv[2 * kk + 2 * tg + 1] = hi2;
          width = (hi2 - lo2) > 1e-15 * fmax(fabs(lo2), fabs(hi2)) + 1e-16 * tnorm + 4.0 * pivmin
                      ? 1.0
                      : 0.0;
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
  if (tid < kk) sv[tid] = fmax(0.5 * (iv[2 * tid] + iv[2 * tid + 1]), 0.0);
  __syncthreads();

  // ---- 3. singular vectors of B from eigenvectors of T_GK
  const double tiny = fmax(2.3e-16 * tnorm, pivmin);
  // the kb vectors of a batch interleaved in lw (entry i of vector t at i kb + t)
  for (int b0 = 0; b0 < k; b0 += kb) {
    const int tv = b0 + tid;
    if (tid < kb && tv < k)
      tgk_vector(tt, n, sv[tv], tiny, tv, half, Y + tv * rows, rows, lw + tid, kb);
    __syncthreads();
  }

  // ---- 4. orthonormalisation.  Vectors of well separated singular values are
  // nearly orthogonal already: two rounds of Cholesky QR (S = Y^T Y = L L^T on
  // the matrix cores, Y <- Y L^{-T}).  A pivot of S below 1e-8 (a tight
  // cluster, or sigma = 0) sends the whole set to classical Gram-Schmidt with
  // reorthogonalisation and repair instead.
  bool cholqr = lwn >= k * k + 2 * k + 1;
  double* const cs = smn >= k * k + 2 * k + 1 ? sm : lw;
  for (int round = 0; round < 2 && cholqr; ++round) {
    double* S = cs;             // k x k, lower triangle becomes L
    double* rdg = cs + k * k;   // 1 / L[t][t]
    double* okf = rdg + k;
    mgemm64(k, k, rows, Y, rows, 1, Y, 1, rows, S, map1(k), map1(1), 1.0, tid, nt);
    __syncthreads();
    if (wave == 0) {
      bool ok = true;
      for (int c = 0; c < k; ++c) {
        const double s2 = S[c * k + c];
        ok = ok && s2 > 1e-8;
        const double piv = sqrt(fmax(s2, 1e-300));
        const double rq = 1.0 / piv;
        wave_sync();
        for (int r = c + 1 + lane; r < k; r += 64) S[r * k + c] *= rq;
        if (lane == 0) {
          S[c * k + c] = piv;
          rdg[c] = rq;
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
    for (int r = tid; r < rows; r += nt) {
      for (int t = 0; t < k; ++t) {
        double z = Y[t * rows + r];
        for (int j = 0; j < t; ++j) z -= Y[j * rows + r] * S[t * k + j];
        Y[t * rows + r] = z * rdg[t];
      }
    }
    __syncthreads();
  }
  double* cf = lw + 8 * n;  // Gram-Schmidt coefficients (k), after the repair scratch
  for (int j = 0; j < k && !cholqr; ++j) {
    double* yj = Y + j * rows;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wave; i < j; i += nw) {
        double s = 0.0;
        for (int r = lane; r < rows; r += 64) s += Y[i * rows + r] * yj[r];
        s = wave_sum(s);
        if (lane == 0) cf[i] = s;
      }
      __syncthreads();
      for (int r = tid; r < rows; r += nt) {
        double v = yj[r];
        for (int i = 0; i < j; ++i) v -= cf[i] * Y[i * rows + r];
        yj[r] = v;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int r = tid; r < rows; r += nt) s += yj[r] * yj[r];
    s = block_sum(s, red, tid, nt);
    if (s < 1e-6) {
      // a tight cluster or a zero singular value: iterate again from other
      // starts with the previous vectors projected out; if the vector still
      // lies in their span, the unit vector with the largest remainder
      // completes the orthonormal set
      if (tid == 0) {
        double t2 = 0.0;
        for (int rep = 0; rep < 3 && t2 <= 1e-6; ++rep) {
          tgk_vector(tt, n, sv[j], tiny, j + 7 * (rep + 1), half, yj, rows, lw, 1);
          for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
              double c = 0.0;
              for (int r = 0; r < rows; ++r) c += Y[i * rows + r] * yj[r];
              for (int r = 0; r < rows; ++r) yj[r] -= c * Y[i * rows + r];
            }
          t2 = 0.0;
          for (int r = 0; r < rows; ++r) t2 += yj[r] * yj[r];
        }
        for (int u = 0; u < rows && t2 <= 1e-6; ++u) {
          for (int r = 0; r < rows; ++r) yj[r] = r == u ? 1.0 : 0.0;
          for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
              double c = 0.0;
              for (int r = 0; r < rows; ++r) c += Y[i * rows + r] * yj[r];
              for (int r = 0; r < rows; ++r) yj[r] -= c * Y[i * rows + r];
            }
          t2 = 0.0;
          for (int r = 0; r < rows; ++r) t2 += yj[r] * yj[r];
          if (t2 < 0.25) t2 = 0.0;
        }
      }
      __syncthreads();
      s = 0.0;
      for (int r = tid; r < rows; r += nt) s += yj[r] * yj[r];
      s = block_sum(s, red, tid, nt);
    }
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int r = tid; r < rows; r += nt) yj[r] *= inv;
    __syncthreads();
  }

  // ---- 5. back-transformation U = H_0 ... H_{nref-1} Y.  Register path
  // (reflectors in rows of W): blocks of bb reflectors, last block first,
  // each applied as I - V T V^T (compact WY form, T upper triangular) through
  // small products on the matrix cores.  Otherwise each wave carries up to
  // four of its vectors through every reflector.
  int bbk = 0;
  if (vrow && nref > 0) {
    for (int b = kMaxWyBlock; b >= 8 && !bbk; b -= 8)
      if ((rows - o) * b + 2 * b * b + 2 * b * k <= lwn) bbk = b;
  }
  if (bbk) {
    double* Vb = lw;  // (rows - i0 - o) x bb
    // VtV (bb x bb) and later W2 (bb x k) share a region; then T (bb x bb,
    // upper) and Wt (bb x k): in sm when they fit, else after V in lw
    const int rw = bbk * (bbk > k ? bbk : k);
    double* VtV = rw + bbk * bbk + bbk * k <= smn ? sm : Vb + (rows - o) * bbk;
    double* W2 = VtV;
    double* Tm = VtV + rw;
    double* Wt = Tm + bbk * bbk;
    const float ik = 1.0f / (float)k;
    for (int i1 = nref; i1 > 0; i1 -= bbk) {
      const int i0 = i1 > bbk ? i1 - bbk : 0, bb = i1 - i0, mb = rows - i0 - o;
      const float ibb = 1.0f / (float)bb;
      // V: column j is reflector i0 + j, zero above its leading 1 (row j)
      for (int q = tid; q < mb * bb; q += nt) {
        int j;
        const int r = qdiv(q, bb, ibb, j);
        Vb[r * bb + j] = r < j ? 0.0 : rp[(i0 + j) * ri + (r - j) * rs];
      }
      __syncthreads();
      mgemm64(bb, bb, mb, Vb, 1, bb, Vb, bb, 1, VtV, map1(bb), map1(1), 1.0, tid, nt);
      mgemm64(bb, k, mb, Vb, 1, bb, Y + i0 + o, 1, rows, Wt, map1(k), map1(1), 1.0, tid, nt);
      __syncthreads();
      // T column by column: T[0:j][j] = -tau_j T[0:j][0:j] VtV[0:j][j].  The
      // sums run over a fixed kMaxWyBlock terms, out-of-range ones masked
      // (their clamped loads stay inside the arrays), so a column's loads
      // issue together.
      if (wave == 0) {
        const int lr = lane < bb ? lane : bb - 1;
        for (int j = 0; j < bb; ++j) {
          const double tj = tq[i0 + j];
          double tij = 0.0;
#pragma unroll
          for (int l = 0; l < kMaxWyBlock; ++l) {
            const int lc = l < bb ? l : bb - 1;
            const double p = Tm[lr * bb + lc] * VtV[lc * bb + j];
            tij += (l >= lane && l < j) ? p : 0.0;
          }
          tij *= -tj;
          wave_sync();
          if (lane < bb) Tm[lane * bb + j] = lane < j ? tij : (lane == j ? tj : 0.0);
          wave_sync();
        }
      }
      __syncthreads();
      // W2 = T Wt (VtV is dead: W2 takes its place)
      for (int q = tid; q < bb * k; q += nt) {
        int tv;
        const int j = qdiv(q, k, ik, tv);
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < kMaxWyBlock; ++l) {
          const int lc = l < bb ? l : bb - 1;
          const double p = Tm[j * bb + lc] * Wt[lc * k + tv];
          acc += (l >= j && l < bb) ? p : 0.0;
        }
        W2[q] = acc;
      }
      __syncthreads();
      // Z = V W2 into the rows of W that hold the reflectors of this block
      // and of the blocks already applied (no longer needed)
      double* Z = W + i0 * rows;
      mgemm64(mb, k, bb, Vb, bb, 1, W2, k, 1, Z, map1(k), map1(1), 1.0, tid, nt);
      __syncthreads();
      for (int q = tid; q < mb * k; q += nt) {
        int tv;
        const int r = qdiv(q, k, ik, tv);
        Y[tv * rows + i0 + o + r] -= Z[q];
      }
      __syncthreads();
    }
  }
  for (int t0 = wave; t0 < k && !bbk; t0 += 4 * nw) {
    const int t1 = t0 + nw, t2 = t0 + 2 * nw, t3 = t0 + 3 * nw;
    double* y0 = Y + t0 * rows;
    double* y1 = Y + (t1 < k ? t1 : t0) * rows;
    double* y2 = Y + (t2 < k ? t2 : t0) * rows;
    double* y3 = Y + (t3 < k ? t3 : t0) * rows;
    for (int i = nref - 1; i >= 0; --i) {
      const double ti = tq[i];
      if (ti == 0.0) continue;
      const int s0i = i + o, len = rows - s0i;
      const double* v = rp + i * ri;
      wave_sync();
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int r = lane; r < len; r += 64) {
        const double vr = v[r * rs];
        s0 += vr * y0[s0i + r];
        s1 += vr * y1[s0i + r];
        s2 += vr * y2[s0i + r];
        s3 += vr * y3[s0i + r];
      }
      s0 = wave_sum(s0) * ti;
      s1 = t1 < k ? wave_sum(s1) * ti : 0.0;
      s2 = t2 < k ? wave_sum(s2) * ti : 0.0;
      s3 = t3 < k ? wave_sum(s3) * ti : 0.0;
      wave_sync();
      for (int r = lane; r < len; r += 64) {
        const double vr = v[r * rs];
        y0[s0i + r] -= s0 * vr;
        if (t1 < k) y1[s0i + r] -= s1 * vr;
        if (t2 < k) y2[s0i + r] -= s2 * vr;
        if (t3 < k) y3[s0i + r] -= s3 * vr;
      }
    }
  }
  __syncthreads();
}

}  // namespace pg
