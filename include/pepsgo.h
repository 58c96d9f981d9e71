/*
 * pepsgo -- per-sample evaluation of a finite open-boundary PEPS on MI355X.
 *
 * Plain C ABI.  Every pointer is a raw host or device address as stated per
 * argument; no HIP or C++ type crosses this interface.  A stream argument is
 * a hipStream_t passed as void* (NULL = the device's default stream).
 *
 * What is computed (Liu, Dong, Han, Guo, He, "Gradient optimization of
 * finite projected entangled pair states", Sec. II):
 *   - W(S), the weight of configuration S (the definition after Eq. (2)):
 *     the single-layer network of fixed-spin slices A_ij = T_ij[s_ij]
 *     (Eq. (1)), contracted by the boundary-MPS method of Fig. 1(d) with the
 *     boundary bond truncated to Dc (zip-up SVD truncation);
 *   - Delta_ij = B_ij / W (Eqs. (4)-(5)) for every site;
 *   - the local energy E(S) = sum_{S'} W(S')/W(S) <S'|H|S> of the J1-J2
 *     Heisenberg model, Eq. (7), with nearest-neighbour (J1) and
 *     plaquette-diagonal next-nearest-neighbour (J2) pairs on the open lattice.
 *
 * Lattice: N rows x M columns; site (i, j) 0-based, rows top to bottom.
 * Tensors: each site T_ij[s][l][r][u][d] (C order), s in [0, d), virtual legs
 * of dimension D except on open edges where they have dimension 1 (Eq. (1)).
 * Packed layout: sites in row-major order, each site contiguous.
 * Configurations: uint8 [batch][N*M] (row-major sites), entries in [0, d);
 * s = 0 is S^z = +1/2.
 *
 * Readings of points the paper leaves open, applied here:
 *   amplitude   psi = <U_{N-2}| row N-1>, the top-down boundary contraction;
 *   gradient    Delta_ij = B_ij / psi_i where psi_i = <U_{i-1}| row i |Dn_{i+1}>
 *               is the exact contraction of row i between its boundary MPSs and
 *               B_ij = d psi_i / d A_ij (so <Delta_ij, A_ij> = 1);
 *   ratios      W(S')/W(S) from shared environments: row sandwiches for
 *               horizontal pairs, exact two-row strips for vertical and
 *               diagonal pairs;
 *   truncation  before a row is absorbed the boundary MPS is made
 *               right-canonical by an exact LQ sweep; each two-column block X
 *               is cut to its chi = min(Dc, rows, cols) leading left singular
 *               vectors.
 *
 * Errors: a negative return code; pepsgo_last_error() describes it.  Checks on
 * arguments and shapes happen before anything is queued.  Numerical trouble
 * in one sample is reported through that sample's flags, never as a failure
 * of the call.
 */
#ifndef PEPSGO_H
#define PEPSGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PEPSGO_VERSION_MAJOR 0
#define PEPSGO_VERSION_MINOR 1

/* status codes */
#define PEPSGO_OK 0
#define PEPSGO_EINVAL (-1)       /* bad argument or shape */
#define PEPSGO_ENOMEM (-2)       /* device allocation failed */
#define PEPSGO_EUNSUPPORTED (-3) /* valid but not supported (size limits, mode) */
#define PEPSGO_EDEVICE (-4)      /* HIP runtime error */
#define PEPSGO_EBUSY (-5)        /* not admitted now (a server's queue is full); retry later */
/* a completed server request (pepsgo_serve_poll) some of whose samples carry
   PEPSGO_F_ZERO_PSI, NONFINITE or NEAR_TIE; the call that launched it did not
   fail.  pepsgo_evaluate itself never returns it: it is asynchronous and the
   flags are per-sample outputs. */
#define PEPSGO_WARN_SAMPLES 1

/* precision of the two-row strip contractions (the vertical and diagonal
   exchange ratios, most of the arithmetic); boundary-MPS truncation, row
   sandwiches (psi, Delta, horizontal ratios) and every log-scale are float64
   in all modes */
#define PEPSGO_FP64 0
#define PEPSGO_FP32 1       /* float32 storage and float32 matrix cores */
#define PEPSGO_BF16_MIXED 2 /* float32 storage; each operand split into three bfloat16
                               pieces, six bfloat16 matrix-core products, float32
                               accumulation (float32-class accuracy) */
#define PEPSGO_BF16 3       /* float32 storage, single bfloat16 operands, float32
                               accumulation: fastest, least accurate */

/* gradient output */
#define PEPSGO_GRAD_NONE 0
#define PEPSGO_GRAD_PER_SAMPLE 1 /* Delta_ij per sample, layout of pepsgo_grad_layout */
#define PEPSGO_GRAD_REDUCED 2    /* the sums of Eq. (3) over the batch instead (no per-sample
                                    Delta leaves the library); needs want_eloc = 1 */

/* per-sample flag bits */
#define PEPSGO_F_ZERO_PSI 1u  /* W(S) = 0 (or a denominator psi_i / strip is 0) */
#define PEPSGO_F_NONFINITE 2u /* a non-finite value appeared */
#define PEPSGO_F_NEAR_TIE 4u  /* a truncation cut between singular values whose
                                 relative gap is <= 1e-8 (kept subspace ill-defined) */
#define PEPSGO_F_REFINED 8u   /* reduced-precision modes: a two-row strip failed its
                                 accuracy check and was recomputed in float64 */

/* size limits of the library */
#define PEPSGO_MAX_SIDE 32 /* N, M <= 32 */
#define PEPSGO_MAX_D 10    /* D <= 10 */
#define PEPSGO_MAX_DC 32   /* Dc <= 32 */

typedef struct pepsgo_ctx_* pepsgo_ctx;
typedef struct pepsgo_peps_* pepsgo_peps;

/* Launch shape of the three main kernels for one (D, Dc, precision): the LDS
   bytes a workgroup may use.  Scratch buffers are placed in LDS in a fixed
   priority order while they fit and in the sample's workspace otherwise, so
   a budget trades LDS-resident intermediates against workgroups per compute
   unit (160 KB of LDS per CU).  0 selects the default. */
typedef struct {
  int zip_lds_bytes;      /* row absorption with truncation */
  int sandwich_lds_bytes; /* row sandwich */
  int strip_lds_bytes;    /* two-row strip */
  int strip_xc;           /* two-row strip: boundary-MPS indices per stage of its column
                             update (1..4; more means fewer barriers, larger intermediates) */
} pepsgo_tuning;

typedef struct {
  int Dc;         /* boundary-MPS cut-off (the paper's D_c1), >= 1 */
  double J1, J2;  /* couplings of Eq. (7) */
  int precision;  /* PEPSGO_FP64, PEPSGO_FP32, PEPSGO_BF16_MIXED or PEPSGO_BF16 */
  int grad_mode;  /* PEPSGO_GRAD_NONE, PEPSGO_GRAD_PER_SAMPLE or PEPSGO_GRAD_REDUCED */
  int want_eloc;  /* 0: skip the local energy (eloc outputs NaN) */
} pepsgo_eval_params;

/* Library version.  Never fails. */
int pepsgo_version(int* major, int* minor);

/* Thread-local description of the last failing call on this thread. */
const char* pepsgo_last_error(void);

/* Bind a context to HIP device `hip_device`.  *out receives the handle.
   Errors: EINVAL (null out, bad device), EDEVICE. */
int pepsgo_create(int hip_device, pepsgo_ctx* out);
/* Release a context (its PEPS handles must be freed first). */
int pepsgo_destroy(pepsgo_ctx ctx);

/* Copy a PEPS into device memory owned by the library (Eq. (1) tensors).
   tensors: float64, packed layout above, host memory if on_device == 0 else
   device memory of the context's device; it is copied and may be reused at
   once.  d must be 2.  Errors: EINVAL (shape), EUNSUPPORTED (limits), ENOMEM. */
int pepsgo_peps_load(pepsgo_ctx ctx, int nrows, int ncols, int d, int D,
                     const double* tensors, int on_device, pepsgo_peps* out);
/* Overwrite the tensors of a loaded PEPS (same shape), e.g. after an
   optimisation step.  Ordered on `stream`. */
int pepsgo_peps_update(pepsgo_peps peps, const double* tensors, int on_device, void* stream);
/* Copy the tensors of a loaded PEPS out (packed layout, nparams doubles), e.g.
   after pepsgo_go_update.  Ordered on `stream`; into host memory
   (on_device == 0) the call returns once the copy is complete.  Errors:
   EINVAL (NULL argument), EDEVICE. */
int pepsgo_peps_read(pepsgo_peps peps, double* tensors, int on_device, void* stream);
/* Free a PEPS handle and its device copy. */
int pepsgo_peps_free(pepsgo_peps peps);

/* Layout of the per-sample gradient block: *elems_per_sample float64 values,
   site (i, j) (k = i*M + j) at offset site_offsets[k], stored [l][r][u][d]
   with that site's dimensions; site_offsets has N*M + 1 entries (the last is
   elems_per_sample).  site_offsets may be NULL. */
int pepsgo_grad_layout(pepsgo_peps peps, int64_t* elems_per_sample, int64_t* site_offsets);

/* Device workspace needed by pepsgo_evaluate for `batch` samples.  A smaller
   workspace (at least the size for one sample) is accepted: the batch is then
   evaluated in chunks that fit. */
int pepsgo_workspace_bytes(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                           size_t* bytes);

/* Evaluate `batch` configurations, asynchronously on `stream`.
   All buffers are device memory of the context's device, owned by the caller:
     configs  uint8  [batch][N*M]
     logabs   double [batch]  ln|psi|      (-inf when flagged ZERO_PSI)
     sign     int8   [batch]  sign of psi  (0 when flagged ZERO_PSI)
     eloc     double [batch]  E(S), total energy (NaN when flagged or want_eloc == 0)
     flags    uint32 [batch]  PEPSGO_F_* bits
     grad     double [batch][elems_per_sample] when grad_mode == PER_SAMPLE
              (NaN block when the sample is flagged ZERO_PSI/NONFINITE);
              double [2 nparams + 3] when grad_mode == REDUCED: the sums of
              pepsgo_go_accumulate over this batch are ADDED to
              grad[0 .. nparams) (sum Delta), grad[nparams .. 2 nparams)
              (sum Delta E) and grad[2 nparams .. 2 nparams + 3) (number of
              samples, sum E, sum E^2), in the packed tensor layout, flagged
              samples left out (zero them before a step's first batch; the
              sums feed pepsgo_go_update directly); else NULL
     workspace  >= the size for one sample (see pepsgo_workspace_bytes)
   No host synchronisation and no allocation happen inside.
   Errors: EINVAL, EUNSUPPORTED (Dc or mode out of range), EDEVICE. */
int pepsgo_evaluate(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                    const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                    uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                    void* stream);

/* pepsgo_evaluate for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same evaluation, with the same results, but its workspace is a fixed
   array of PEPSGO_NOALLOC_SCRATCH_BYTES that the library keeps in device
   memory (one per device, held until the process ends) instead of a caller
   buffer.  The call allocates nothing.  Batches whose workspace exceeds the
   array are evaluated in chunks through it; a shape of which one sample
   alone needs more (see pepsgo_workspace_bytes with batch = 1) is refused
   with EUNSUPPORTED.  The array keeps the previous call's contents; nothing
   in it needs to start at zero (every sample's state is initialised by the
   first kernel).  All calls on one device share the array: calls that
   overlap in time on one device (different streams or threads) race, so the
   caller serialises them.  Arguments and other errors as pepsgo_evaluate. */
#define PEPSGO_NOALLOC_SCRATCH_BYTES (128u << 20)
int pepsgo_evaluate_noalloc(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                            const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                            uint32_t* flags, double* grad, void* stream);

/* One Metropolis step per chain, on the device (the sampling of the paper,
   Sec. II: configurations drawn with weight W(S)^2).  Evaluates the current
   configurations exactly as pepsgo_evaluate does (outputs for the states
   before the move; params->want_eloc must be 1), then for sample b proposes
   exchanging the two spins of nearest-neighbour bond bonds[b] and accepts
   with probability min(1, R^2), R = W(S')/W(S) being the exchange ratio the
   local energy of S already used (row sandwich for a horizontal bond, two-row
   strip for a vertical one), when uniforms[b] < min(1, R^2).  A bond whose
   spins agree, or a flagged sample, does not move.  Accepted exchanges are
   applied to `configs` in place.
     configs   uint8 [batch][N*M], device, read and updated
     bonds     int32 [batch], device: horizontal bonds (i, j)-(i, j+1) are
               numbered i*(M-1) + j, vertical (i, j)-(i+1, j) N*(M-1) + i*M + j;
               values outside [0, N*(M-1) + (N-1)*M) propose nothing
     uniforms  double [batch], device, in [0, 1)
     accepted  uint8 [batch], device: 1 where the exchange was applied
   The other arguments as pepsgo_evaluate.  Errors: as pepsgo_evaluate,
   EINVAL when want_eloc == 0. */
int pepsgo_metropolis_step(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                           uint8_t* configs, const int32_t* bonds, const double* uniforms,
                           uint8_t* accepted, double* logabs, int8_t* sign, double* eloc,
                           uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                           void* stream);

/* One Metropolis sweep per chain, on the device (the sampling with weight
   W(S)^2 of Sec. II, in sweeps): every nearest-neighbour bond is visited once,
   row by row from the top: the horizontal bonds (i, j)-(i, j+1), j = 0..M-2,
   then (for i < N-1) the vertical bonds (i, j)-(i+1, j), j = 0..M-1.  Bond k
   of that order (row i's horizontal bonds start at k = i (2M - 1), its
   vertical ones M - 1 later) with unequal spins has its exchange accepted when
   uniforms[b][k] < min(1, R^2), R = W(S')/W(S) from the shared environments
   of the configuration as it stands (the row-i sandwich for a horizontal
   bond, the strip of rows i, i+1 for a vertical one, as in the local energy);
   R is the ratio of the two contractions that differ in the exchanged
   column(s) only.  Environments are reused: the bottom ones are built once
   per sweep, U_{i-1} once per row from the rows as they stand, and along a
   row (strip) the right environments once, the left one column by column.
   One sweep costs about one evaluation.  Decisions are float64 whatever
   params->precision says; J1, J2 and grad_mode are ignored.
     configs   uint8 [batch][N*M], device, updated in place
     uniforms  double [batch][nbonds], device, in [0, 1); nbonds = N(M-1) + (N-1)M
     accepted  uint8 [batch][nbonds], device: 1 where the exchange was applied
     ratios    double [batch][nbonds], device, or NULL: R of each proposed
               bond (NaN where the spins were equal or the sample stopped)
     workspace as for pepsgo_evaluate with want_eloc = 1 and precision FP64
   A sample whose environments vanish or stop being finite stops moving.
   Errors: EINVAL (NULL buffer, workspace too small), EUNSUPPORTED (Dc),
   EDEVICE. */
int pepsgo_metropolis_sweep(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                            uint8_t* configs, const double* uniforms, uint8_t* accepted,
                            double* ratios, void* workspace, size_t workspace_bytes,
                            void* stream);

/* Simple-update imaginary-time evolution, the initialiser of Sec. III.
   The state is held by the caller as
     gamma    double, device, the packed tensor layout of the loaded PEPS
              (site tensors Gamma_ij[s][l][r][u][d])
     lambdas  double, device, [nbonds][D] weight vectors, bond b = i*(M-1)+j
              for (i,j)-(i,j+1) and N*(M-1) + i*M + j for (i,j)-(i+1,j)
              (all ones for a fresh start)
   and represents the PEPS whose tensors are Gamma with sqrt(lambda) on both
   sides of every bond.  One step applies exp(-dtau J1 S_a.S_b) to every
   nearest-neighbour bond (J2 terms are not evolved), in the groups:
   horizontal bonds with j even, j odd, vertical bonds with i even, i odd
   (bonds of a group share no site), each followed by an SVD cut back to D
   computed from the QR factors of the two site tensors (cost O(D^5) per
   bond); the new weights are the kept singular values over their 2-norm,
   and dividing a weight out skips entries <= 1e-12 of the bond's largest.
   su_evolve runs nsteps steps in place, asynchronously on `stream`, with a
   caller-owned device workspace of pepsgo_su_workspace_bytes.
   su_to_peps writes the absorbed tensors into the loaded PEPS (for
   pepsgo_evaluate and the gradient steps).
   Errors: EINVAL (NULL argument, nsteps < 0, non-finite J1/dtau, workspace
   too small), EDEVICE. */
int pepsgo_su_workspace_bytes(pepsgo_peps peps, size_t* bytes);
int pepsgo_su_evolve(pepsgo_peps peps, double* gamma, double* lambdas, double J1, double dtau,
                     int nsteps, void* workspace, size_t workspace_bytes, void* stream);
int pepsgo_su_to_peps(pepsgo_peps peps, const double* gamma, const double* lambdas, void* stream);
/* The D-ramp of Sec. III (start at a small D, then use the converged tensors
   at a larger one): writes the state (gamma, lambdas) of handle `from` at the
   bond dimension of handle `to` (same lattice and device, D_to >= D_from)
   into gamma_out / lambdas_out (device, the layouts above for `to`), every
   inner leg and weight vector padded with zeros.  The represented state is
   unchanged; later steps at D_to fill the new bond space.  Asynchronous on
   `stream`.  Errors: EINVAL (NULL argument, shapes), EDEVICE. */
int pepsgo_su_pad(pepsgo_peps from, const double* gamma, const double* lambdas, pepsgo_peps to,
                  double* gamma_out, double* lambdas_out, void* stream);

/* Measurement helper (not part of the method): one launch of a throughput
   probe on `stream`, to confirm on the device the peaks a roofline divides
   by.  kind: PEPSGO_PROBE_FMA64 (float64 vector FMA chains),
   PEPSGO_PROBE_MFMA64 / MFMA32 / MFMA_BF16 (16x16x4 float64, 16x16x4
   float32, 16x16x16 bfloat16 matrix-core instructions, the ones the strips
   and sandwiches use).  `blocks` workgroups of 256 threads each run `iters`
   rounds of independent chains; *flops receives the launch's flop count
   (2 per multiply-add) at once, the caller times the launch (events on
   `stream`).  sink: device, >= blocks doubles (written only to keep the
   chains live).  Errors: EINVAL, EDEVICE. */
#define PEPSGO_PROBE_FMA64 0
#define PEPSGO_PROBE_MFMA64 1
#define PEPSGO_PROBE_MFMA32 2
#define PEPSGO_PROBE_MFMA_BF16 3
int pepsgo_peak_probe(int kind, int blocks, int iters, double* sink, double* flops, void* stream);

/* Spin-spin correlations and m_s^2(k) on a window of the lattice (Sec. IV:
   the paper sums over the central (L-2)^2 or (L-4)^2 sites).
   sz_counts adds, over the `batch` configurations (device, [batch][nrows*ncols])
   drawn with weight W^2, for every pair (p, q) of the h x w window with corner
   (r0, c0) (window sites row-major, p = a*w + b for site (r0+a, c0+b)):
     same[p*h*w + q] += number of samples with s_p = s_q      (int64, device)
     nsamples[0]     += number of samples counted             (int64, device)
   skipping samples flagged ZERO_PSI or NONFINITE when `flags` (device,
   [batch]) is given; NULL counts every sample.  Exact integer counts, so the
   result is independent of chunking and order.  <S^z_p S^z_q> =
   (2 same - n) / (4 n).
   structure_factor writes out[0] (device) = factor / (h w)^2 *
   sum_pq <S^z_p S^z_q> cos(kx (x_p - x_q) + ky (y_p - y_q)) with x the column
   and y the row within the window; factor = 3 gives m_s^2(k) of a
   spin-rotation-invariant state (<S_p . S_q> = 3 <S^z_p S^z_q>), and
   k = (pi, pi) the staggered magnetisation M^2.  NaN when no sample was
   counted.  The transverse part of <S_p . S_q> comes from pepsgo_transverse
   below.  Both are asynchronous on `stream`.
   Errors: EINVAL (window outside the lattice, NULL buffer), EDEVICE. */
int pepsgo_sz_counts(int nrows, int ncols, int r0, int c0, int h, int w, int batch,
                     const uint8_t* configs, const uint32_t* flags, int64_t* same,
                     int64_t* nsamples, void* stream);
int pepsgo_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples, double kx,
                            double ky, double factor, double* out, void* stream);

/* Transverse part of <S_p . S_q> on the same window (Sec. IV, m_s^2(k) sums
   <S_i . S_j> = <S^z_i S^z_j> + <S^+_i S^-_j + S^-_i S^+_j>/2 over the window
   pairs).  Over configurations drawn with weight W^2 its local value is
   O_pq(S) = 1/2 [s_p != s_q] R_pq with R_pq = W(S^{pq})/W(S) (spins at p and q
   exchanged), and O_pp = 1/2.  R_pq for p in row a, q in row b >= a (p before
   q row-major): rows a..b-1 of S^{pq} zipped top-down (truncation to Dc) into
   U_{a-1}(S), closed by the exact row-b sandwich with Dn_{b+1}(S), divided by
   psi_b(S) = <U_{b-1}(S)| row b |Dn_{b+1}(S)>: both share the environments of
   the rows that do not change (for b = a, the horizontal ratio of E(S)).
   Float64 throughout; of `params` only Dc is used.
   configs  device [batch][nrows*ncols] spin labels.
   ratios   optional device [batch][n][n] float64 out (n = h w, window sites
            row-major): R_pq, symmetric, NaN on the diagonal, where s_p = s_q
            and for samples flagged ZERO_PSI or NONFINITE.
   sums     device [n*n] float64, added to: sum over counted samples of O_pq.
   count    device [1] int64, added to: samples counted (those not flagged
            ZERO_PSI or NONFINITE).
   flags    device [batch] uint32 out: PEPSGO_F_ZERO_PSI / NONFINITE of the
            sample's own environments, NONFINITE when a counted ratio is not
            finite, NEAR_TIE when a truncation of the sample or of one of its
            exchanged configurations met a near tie (counted all the same).
   Cost: h w exchanged configurations per sample, each zipped through the
   window rows below its first site.  The workspace (device, caller-owned)
   holds any number of samples of transverse_workspace_bytes(batch = 1); a
   smaller one than `batch` needs is used in chunks.  The sums are
   independent of chunking and timing (each pair adds its samples in order).
   Asynchronous on `stream`.  Errors: EINVAL (NULL argument, window outside
   the lattice, workspace below one sample), EUNSUPPORTED (window above
   PEPSGO_MAX_WINDOW sites, parameters out of range), EDEVICE. */
#define PEPSGO_MAX_WINDOW 1024
int pepsgo_transverse_workspace_bytes(pepsgo_peps peps, const pepsgo_eval_params* params, int r0,
                                      int c0, int h, int w, int batch, size_t* bytes);
int pepsgo_transverse(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                      const uint8_t* configs, int r0, int c0, int h, int w, double* ratios,
                      double* sums, int64_t* count, uint32_t* flags, void* workspace,
                      size_t workspace_bytes, void* stream);

/* m_s^2(k) of Sec. IV from both parts: out[0] (device) = 1/(h w)^2 *
   sum_pq <S_p . S_q> cos(kx (x_p - x_q) + ky (y_p - y_q)) with
   <S_p . S_q> = (2 same - n)/(4 n) + trans[p*h*w + q] / ntrans[0]
   (same, n from pepsgo_sz_counts; trans, ntrans from pepsgo_transverse).
   NaN when either count is 0.  Asynchronous on `stream`.
   Errors: EINVAL (window size, NULL buffer), EDEVICE. */
int pepsgo_spin_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples,
                                 const double* trans, const int64_t* ntrans, double kx, double ky,
                                 double* out, void* stream);

/* Gradient optimisation (Sec. II): Eq. (3), dE/dA = 2<Delta E> - 2<Delta><E>
   over configurations drawn with weight W^2, and the sign update of Eq. (6).
   go_accumulate adds, over the `batch` samples of one evaluation (its device
   outputs grad [batch][elems_per_sample], eloc, flags and the configurations
   it evaluated), into caller-owned device sums laid out like the packed
   tensors of pepsgo_peps_load:
     sum_delta[q]    += sum_S Delta_q(S)         (Delta of S belongs to the
     sum_delta_e[q]  += sum_S Delta_q(S) E(S)     slice T_ij[s_ij] of its spin)
     stats[0..2]     += (number of samples, sum E, sum E^2)
   skipping samples flagged ZERO_PSI or NONFINITE; zero the sums before the
   first batch of a step.  go_update then moves every tensor element of the
   loaded PEPS, in place on the device:
     T_q <- T_q - p_q dt sign(2 sum_delta_e_q / n - 2 (sum_delta_q / n)(sum E / n))
   with p_q in [0, 1] supplied per element (device, packed layout) and
   sign(0) = 0; nothing moves while n = 0.  Both are asynchronous on `stream`.
   Errors: EINVAL (NULL argument, dt < 0), EDEVICE. */
int pepsgo_go_accumulate(pepsgo_peps peps, int batch, const uint8_t* configs, const double* grad,
                         const double* eloc, const uint32_t* flags, double* sum_delta,
                         double* sum_delta_e, double* stats, void* stream);
int pepsgo_go_update(pepsgo_peps peps, const double* sum_delta, const double* sum_delta_e,
                     const double* stats, double dt, const double* p, void* stream);

/* A whole evaluation captured as one HIP graph.  graph_create records the
   launch sequence of pepsgo_evaluate with exactly these arguments (same
   buffers, batch and parameters, and the tuning in use) without running it;
   graph_launch replays it on `stream` -- e.g. once per sweep of Markov
   chains whose configuration buffer stays resident and is rewritten in place
   between replays.  The buffers must outlive the graph.  Replays on one
   stream are ordered; replays of one graph must not overlap.
   Errors: as pepsgo_evaluate (batch >= 1), EDEVICE for capture failures. */
typedef struct pepsgo_graph_* pepsgo_graph;
int pepsgo_graph_create(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                        const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                        uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                        pepsgo_graph* out);
int pepsgo_graph_launch(pepsgo_graph graph, void* stream);
int pepsgo_graph_free(pepsgo_graph graph);

/* Tuning table of a context, keyed by (D, Dc, precision).  get returns the
   entry in use (the defaults when none was set); set replaces it (NULL
   removes it).  The workspace size of pepsgo_workspace_bytes follows the
   entry in use, so query it after tuning. */
int pepsgo_tune_get(pepsgo_ctx ctx, int D, int Dc, int precision, pepsgo_tuning* out);
int pepsgo_tune_set(pepsgo_ctx ctx, int D, int Dc, int precision, const pepsgo_tuning* t);

/* Autotuner: time every candidate LDS budget of each kernel class on `batch`
   device configurations of this PEPS with these parameters (one evaluation
   per candidate row, each class timed with events on `stream`), keep the
   fastest per class in the context's table and return it in *chosen (may be
   NULL).  Allocates its own outputs and workspace for the run and frees them;
   synchronises the stream; resets the profiling counters.
   Errors: as pepsgo_evaluate, ENOMEM. */
int pepsgo_autotune(pepsgo_peps peps, const pepsgo_eval_params* params, int batch,
                    const uint8_t* configs, void* stream, pepsgo_tuning* chosen);

/* Save / load the tuning table as text ("D Dc precision zip sandwich strip
   strip_xc" per line after a header naming the device architecture); load
   skips a file written for another architecture and returns the entries read
   (>= 0). */
int pepsgo_tune_save(pepsgo_ctx ctx, const char* path);
int pepsgo_tune_load(pepsgo_ctx ctx, const char* path);

/* Kernel classes reported by pepsgo_profile_read. */
#define PEPSGO_K_EDGES 0    /* first/last rows read as boundary MPSs */
#define PEPSGO_K_ZIP 1      /* row absorption with LQ sweep and SVD truncation */
#define PEPSGO_K_SANDWICH 2 /* row sandwich: psi_i, Delta_ij, horizontal ratios */
#define PEPSGO_K_STRIP 3    /* two-row strip: vertical and diagonal ratios */
#define PEPSGO_K_FINALIZE 4 /* local-energy assembly and outputs */
#define PEPSGO_K_COUNT 5

/* Observability: when enabled, every kernel launched by pepsgo_evaluate on
   this context is bracketed by HIP events on its stream; pepsgo_profile_read
   waits for those events and returns the summed device time (ms) and launch
   count of one kernel class since the last reset.  enable: 1 on, 0 off,
   -1 reset counters (keeps the current state). */
int pepsgo_profile(pepsgo_ctx ctx, int enable);
int pepsgo_profile_read(pepsgo_ctx ctx, int kernel_class, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * The Monte Carlo estimates of the paper (Sec. II: E and its gradient as
 * averages over configurations drawn with weight W^2) consume evaluations
 * of many independent batches; a server takes such batches as requests for
 * any loaded PEPS and any parameters, and keeps the device busy with them:
 *   - a request is split into chunks of at most max_chunk samples; chunks
 *     are the unit of admission and run on `streams` device streams at once,
 *     so requests that arrive while others run are started as soon as a
 *     stream and memory free up, and their kernels overlap on the device;
 *   - each chunk's workspace comes from one device pool reserved at creation
 *     (pool_bytes): a chunk is admitted only when its footprint fits, and is
 *     halved (down to min_chunk samples) when the pool is short;
 *   - a chunk may gather samples of several pending requests with the same
 *     PEPS and parameters into one launch (their configurations are copied
 *     into the pool and the results copied back);
 *   - the next free stream goes to the pending request with the fewest
 *     chunks in flight, earliest arrival first among equals.
 * Every sample is computed by the same kernels with the same arithmetic
 * whatever chunk it lands in, so a result does not depend on the mix.
 * The server owns a thread that launches, polls and completes the work; the
 * PEPS handles used by pending requests must stay loaded and unchanged.
 * ------------------------------------------------------------------------ */
typedef struct pepsgo_server_* pepsgo_server;

typedef struct {
  size_t pool_bytes; /* device memory reserved for chunk workspaces and staging
                        (0: 4 GiB) */
  int streams;       /* chunks in flight at once, 1..16 (0: 4) */
  int max_chunk;     /* samples per launch, >= 1 (0: 2048) */
  int min_chunk;     /* smallest chunk when the pool is short (0: 32) */
  int max_pending;   /* requests queued or running at most; a submit beyond it
                        returns PEPSGO_EBUSY (0: no limit) */
} pepsgo_serve_config;

typedef struct {
  uint64_t id;         /* as returned by pepsgo_serve_submit */
  int status;          /* PEPSGO_OK; PEPSGO_WARN_SAMPLES when some of its samples are
                          flagged ZERO_PSI, NONFINITE or NEAR_TIE; or the error of a
                          launch of this request */
  int batch;
  int64_t t_submit_ns; /* host steady clock at submission */
  int64_t t_start_ns;  /* first chunk launched */
  int64_t t_done_ns;   /* completion of the last chunk observed by the server */
} pepsgo_serve_done;

/* Start a server on the context's device.  Errors: EINVAL, ENOMEM (pool), EDEVICE. */
int pepsgo_serve_create(pepsgo_ctx ctx, const pepsgo_serve_config* cfg, pepsgo_server* out);

/* Queue one request.  Buffers as for pepsgo_evaluate (device memory owned by
   the caller, left untouched until the request completes); no workspace is
   passed.  Returns at once; *id identifies the request in completions.
   Errors (checked before queueing): EINVAL, EUNSUPPORTED, EINVAL when one
   sample's footprint exceeds the pool, EBUSY (nothing queued) when
   max_pending requests are already queued or running. */
int pepsgo_serve_submit(pepsgo_server srv, pepsgo_peps peps, const pepsgo_eval_params* params,
                        int batch, const uint8_t* configs, double* logabs, int8_t* sign,
                        double* eloc, uint32_t* flags, double* grad, uint64_t* id);

/* Collect up to `max` completed requests into out[], waiting up to
   timeout_us microseconds for the first one (0: do not wait).  Returns the
   number collected (>= 0) or an error code.  Results of a completed request
   are in its buffers when it is returned here. */
int pepsgo_serve_poll(pepsgo_server srv, pepsgo_serve_done* out, int max, int64_t timeout_us);

/* Requests queued or running. */
int pepsgo_serve_pending(pepsgo_server srv, int* requests);

/* Service figures over the requests completed since creation (or since the
   last reset): request and sample counts, request latency (submission to
   completion) at the 50th and 99th percentiles over the last 65536 requests,
   and samples per second of wall time from the first submission to the last
   completion.  reset != 0 starts a new period after reading. */
typedef struct {
  int64_t requests;
  int64_t samples;
  double p50_ms, p99_ms;
  double samples_per_s;
  int pending; /* queued or running now */
} pepsgo_serve_stats_t;
int pepsgo_serve_stats(pepsgo_server srv, pepsgo_serve_stats_t* out, int reset);

/* Finish every queued request, stop the thread and release the pool and
   streams.  Completions not yet polled are discarded. */
int pepsgo_serve_destroy(pepsgo_server srv);

#ifdef __cplusplus
}
#endif

#endif /* PEPSGO_H */
