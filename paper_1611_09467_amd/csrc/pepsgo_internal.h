// Internal structures shared by the kernels and the host side of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pepsgo.h"

namespace pg {

constexpr int kMaxSide = PEPSGO_MAX_SIDE;
constexpr int kThreads = 256;     // workgroup size of the per-sample kernels
constexpr int kZipThreads = 256;  // workgroup size of the truncation kernel
constexpr int kRedDoubles = 64;   // reduction scratch (one slot per wave)
constexpr uint32_t kFlagZero = PEPSGO_F_ZERO_PSI;
constexpr uint32_t kFlagNonfinite = PEPSGO_F_NONFINITE;
constexpr uint32_t kFlagNearTie = PEPSGO_F_NEAR_TIE;
constexpr uint32_t kFlagRefined = PEPSGO_F_REFINED;
// reduced-precision strips: a strip is recomputed in float64 when the left /
// right environment overlap strays from the strip value by more than
// kRefineMaxDev (relative) at some cut, or when that deviation times the sum
// of |ratio terms| of the strip exceeds its share (1 of N-1 strips) of an
// energy error of kRefineTolSite per site
constexpr double kRefineMaxDev = 1e-3;
constexpr double kRefineTolSite = 1e-4;
constexpr double kNearTieRelGap = 1e-8;
constexpr double kNegligibleRelSv = 1e-13;

// Where each scratch buffer of a kernel lives: byte offset into LDS, or into
// the sample's global scratch region when bit b of glob is set.
constexpr int kMaxBufs = 16;
struct BufPlan {
  int64_t off[kMaxBufs];  // in doubles
  uint32_t glob;
};

// Everything a kernel needs to find its sample's data.
struct Lat {
  int N, M, D, Dc, chimax;
  const double* T;          // packed tensors
  const int64_t* site_off;  // [N*M] offset of site k in T (doubles)
  const uint8_t* cfg;       // [batch][N*M] (this chunk)
  double* ws;               // workspace base of this chunk
  int64_t ws_stride;        // doubles per sample
  int64_t off_env;          // first MPS slot
  int64_t env_stride;       // doubles per MPS slot (M site slots)
  int64_t site_slot;        // doubles per site slot
  int64_t off_envlog;       // [n_env] log-scales
  int64_t off_rowlog;       // [N] ln|psi_i|
  int64_t off_rowsign;      // [N] sign psi_i (as double)
  int64_t off_eloc;         // [1] off-diagonal energy accumulator
  int64_t off_flags;        // [0] flags (uint32 in a double slot), [1] strip redo marker,
                            // [2] exchange ratio of the proposed Metropolis bond
  int64_t off_re;           // sandwich right environments, (M+1) slots
  int64_t re_slot;
  int64_t off_re2;          // strip right environments, (M+1) slots
  int64_t re2_slot;
  int64_t off_scratch;      // global-placed kernel scratch
  double J1, J2;
  double* grad;             // output gradient base for this chunk (or null)
  int64_t grad_stride;
  const int64_t* grad_off;  // [N*M]
  const double* ones;       // device array of 1.0 (trivial environments)
  const int32_t* mbond;     // [batch] Metropolis: proposed bond per sample (this chunk), or null
};

__host__ __device__ inline void site_dims(int N, int M, int D, int i, int j, int* dl, int* dr,
                                          int* du, int* dd) {
  *dl = j == 0 ? 1 : D;
  *dr = j == M - 1 ? 1 : D;
  *du = i == 0 ? 1 : D;
  *dd = i == N - 1 ? 1 : D;
}

// Shape of one zip (absorption of a row into a boundary MPS).
struct ZipShape {
  int row;  // lattice row absorbed
  int dir;  // 0: from above (contract u, new physical leg d); 1: from below
  int in_slot, out_slot, tmp_slot;
  int chi_in[kMaxSide + 1];  // bonds of the input MPS
  int chic[kMaxSide + 1];    // bonds after the exact LQ sweep
  int nb[kMaxSide + 1];      // bonds of the output MPS
  int eig_batch;             // inverse iterations run together (scratch size)
  int lw_doubles;            // size of the truncation's scratch buffer ZB_LW
  int c_doubles;             // size of the carry buffer ZB_C (idle during the truncation)
  int threads;               // workgroup size: 256 (four waves) or 64 (one wave)
};

// Shape of a row sandwich <U_{i-1}| row i |Dn_{i+1}>.
struct SandShape {
  int row;
  int top_slot, bot_slot;  // -1: trivial
  int ta[kMaxSide + 1], tb[kMaxSide + 1];
  int want_grad, want_eloc;
};

// Shape of a strip <U_{i-1}| rows i, i+1 |Dn_{i+2}>.
struct StripShape {
  int row;
  int top_slot, bot_slot;
  int ta[kMaxSide + 1], tb[kMaxSide + 1];
  int want_diag;
  int refine;  // 1: float64 pass over the samples whose reduced-precision strip was rejected
  int xc;      // x values per stage of the column update (slots of the intermediates)
};

// One row of the transverse-correlation pass over the instances (window site
// p, sample r) of a chunk: the single-flip values of row `row` of S^p.
struct FlipShape {
  int row;
  int top_slot;  // instance slot holding the top environment, -1: trivial
  int bot_slot;  // slot of Dn_{row+1} in the sample's own workspace, -1: trivial
  int ta[kMaxSide + 1], tb[kMaxSide + 1];
  int r0, c0, h, w;  // the window
  int nbr;           // samples of the chunk (instance v = x * nbr + r)
  int64_t off_rat;   // instance workspace: its ratios to later window sites (h w doubles)
};

// host helpers shared by the C-ABI sources (pepsgo_capi.cpp)
int api_fail(int code, const char* fmt, ...);  // record the thread's last error, return code
int ctx_device(pepsgo_ctx c);
void peps_shape(pepsgo_peps p, int* N, int* M);

// kernel launchers (pepsgo_kernels.hip)
hipError_t launch_edges(const Lat& L, int nb, int slot_top0, int slot_bot, int reset,
                        hipStream_t s);
hipError_t launch_sweep_row(const Lat& L, const SandShape& z, const BufPlan& p, int lds, int nb,
                            uint8_t* cfg, const double* uniforms, uint8_t* accepted,
                            double* ratios, int nbonds, int k0, hipStream_t s);
hipError_t launch_sweep_strip(const Lat& L, const StripShape& z, const BufPlan& p, int lds,
                              int nb, uint8_t* cfg, const double* uniforms, uint8_t* accepted,
                              double* ratios, int nbonds, int k0, hipStream_t s);
hipError_t launch_sweep_clear(int64_t n, uint8_t* accepted, double* ratios, hipStream_t s);
hipError_t launch_zip(const Lat& L, const ZipShape& z, const BufPlan& p, int lds_bytes, int nb,
                      hipStream_t s);
hipError_t launch_sandwich(const Lat& L, const SandShape& z, const BufPlan& p, int lds_bytes,
                           int nb, hipStream_t s);
hipError_t launch_strip(const Lat& L, const StripShape& z, const BufPlan& p, int lds_bytes,
                        int nb, int precision, hipStream_t s);
hipError_t prepare_lds(int lds_zip, int lds_sand, int lds_strip, int precision);
// device address of the fixed workspace of pepsgo_evaluate_noalloc on the current device
hipError_t scratch_address(void** ptr);
int64_t su_workspace_doubles(int N, int M, int D);
hipError_t launch_su_step(int N, int M, int D, double* G, const int64_t* site_off, double* lam,
                          double* ws, const double* gate, hipStream_t s);
hipError_t launch_su_pad(int N, int M, int Df, int Dt, const int64_t* off_f, const int64_t* off_t,
                         int64_t nparams_t, const double* Gf, double* Gt, const double* lamf,
                         double* lamt, hipStream_t s);
hipError_t launch_su_absorb(int N, int M, int D, const double* G, const int64_t* site_off,
                            const double* lam, int64_t nparams, double* T, hipStream_t s);
hipError_t launch_sz_counts(int N, int M, int r0, int c0, int h, int w, int batch,
                            const uint8_t* cfg, const uint32_t* flags, int64_t* same,
                            int64_t* nsamples, hipStream_t s);
hipError_t launch_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples,
                                   const double* trans, const int64_t* ntrans, double kx,
                                   double ky, double factor, double* out, hipStream_t s);
hipError_t launch_flags_or(const uint32_t* f, int n, uint32_t* out, hipStream_t s);
hipError_t launch_corr_init(const Lat& V, const FlipShape& z, int nv, const uint8_t* cfg_real,
                            uint8_t* cfg_inst, hipStream_t s);
hipError_t launch_corr_copy(const Lat& V, const Lat& R, int nbr, int v0, int count, int src_slot,
                            int dst_slot, hipStream_t s);
hipError_t launch_flip_row(const Lat& V, const Lat& R, const FlipShape& z, const BufPlan& p,
                           int lds, int nv, hipStream_t s);
hipError_t launch_corr_finish(const Lat& V, const Lat& R, const FlipShape& z, uint32_t* flags,
                              double* ratios, double* sums, int64_t* count, hipStream_t s);
hipError_t launch_go_accumulate(int batch, int nsites, int64_t gel, int64_t grad_stride,
                                const uint8_t* cfg, const double* grad, const double* eloc,
                                const uint32_t* flags, const int64_t* grad_off,
                                const int64_t* site_off, double* sd, double* sde, double* stats,
                                hipStream_t s);
hipError_t launch_go_update(int64_t nparams, double* T, const double* sd, const double* sde,
                            const double* stats, double dt, const double* p, hipStream_t s);
hipError_t launch_metropolis(const Lat& L, int nb, const double* uniforms, uint8_t* cfg,
                             uint8_t* accepted, hipStream_t s);
hipError_t launch_finalize(const Lat& L, int nb, int want_eloc, double* logabs, int8_t* sign,
                           double* eloc, uint32_t* flags, hipStream_t s);

// buffer lists (sizes in doubles) of each kernel, in LDS priority order
enum ZipBuf { ZB_RED, ZB_G, ZB_V, ZB_X, ZB_C, ZB_LW, ZB_MISC, ZB_COUNT };
enum SandBuf { SB_RED, SB_T1, SB_T2, SB_LE0, SB_LE1, SB_E1, SB_E2, SB_Q, SB_STG, SB_COUNT };
enum StripBuf { TB_RED, TB_T1, TB_T2, TB_STG, TB_LE0, TB_LE1, TB_E1, TB_E2, TB_COUNT };

}  // namespace pg
