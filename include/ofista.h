/*
 * ofista.h -- C ABI of the MI355X (gfx950) Online FISTA library, libofista.so.
 *
 * Online FISTA (Flynn, Ivanov, Yazici, "Online Sparse Synthetic Aperture Radar
 * Imaging") reconstructs a sparse SAR scene pulse by pulse.  For every received
 * pulse d_s it forms the per-pulse forward operator A_s = F_s W (Section III-A,
 * eq. for G), folds it into the running sufficient statistics
 * H += A_s^H A_s and b += A_s^H d_s (Section III-C, the Delta-A / Delta-b and
 * A_n / b_n equations; the paper's A_n is called H here), picks the step
 * tau = 1/L_n (Section III-B spectral-norm condition and the incremental bound
 * of Section III-C), and runs m warm-started FISTA steps (Algorithm 1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Complex values are complex64: two consecutive floats (re, im).
 * - Pixels form an n_x by n_y grid on the plane z = 0; pixel (iy, ix) sits at
 *   (x0 + ix*dx, y0 + iy*dy, 0) and has flat index i = iy*n_x + ix; N = n_x*n_y.
 * - The sparse coefficients c (length M) are the dictionary's: M = N with the
 *   same flat index for IDENTITY and HAAR2D; M is the atom count for EDGELET
 *   (ofista_coef_count).  H is M x M, b and every coefficient vector have M
 *   entries; images and scenes have N.
 * - The kernel of F_s is exp(-i 4 pi f_k R_{s,i} / c0) with R the Euclidean
 *   distance between platform position s and pixel i and f_k = freq0 + k*dfreq
 *   (the Section II phase with amplitude 1, on a stepped-frequency grid).
 *   Range and phase are evaluated in FP64 on the device.
 * - Device pointers ("d_" prefix) must point to device memory of the device
 *   that was current at ofista_create; host pointers are plain host memory.
 * - Every call that takes a ctx enqueues its device work on the stream given
 *   to ofista_create and returns without waiting, unless stated otherwise.
 * - A ctx is single-threaded: calls on one ctx must not overlap.
 * - ofista_reset, ofista_push_pulse (without validate_input and without
 *   recording, whose checkpoints synchronise),
 *   ofista_reconstruct (launch-pair step kernel; either storage, any
 *   dictionary) and ofista_reconstruct_static (GRAM storage) enqueue kernels
 *   and device-to-device copies only: no host
 *   synchronisation and no memset, so a sequence of them can be captured from
 *   the ctx's stream into a HIP graph and replayed.  The host side of the ctx
 *   (pulse count, step parity, momentum t) advances when the calls are made,
 *   not when the graph replays: begin a captured sequence with ofista_reset,
 *   and make no other state-changing call on the ctx between replays.
 * - Errors are returned as ofista_status; nothing throws or aborts across the
 *   ABI.  After OFISTA_E_HIP the ctx is poisoned and every later call on it
 *   returns OFISTA_E_STATE (ofista_destroy still works).
 */
#ifndef OFISTA_H
#define OFISTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque context of one reconstruction (host memory owned by the library). */
struct ofista_ctx;

typedef enum ofista_status {
  OFISTA_OK = 0,
  OFISTA_E_ARG = -1,         /* null pointer, bad size or enum value         */
  OFISTA_E_RANGE = -2,       /* pulse index outside [0, n_pos)               */
  OFISTA_E_STATE = -3,       /* call not valid now (e.g. no pulse yet), or
                                the ctx is poisoned by an earlier HIP error  */
  OFISTA_E_WORKSPACE = -4,   /* workspace null, misaligned or too small      */
  OFISTA_E_UNSUPPORTED = -5, /* valid but unsupported combination            */
  OFISTA_E_HIP = -6          /* a HIP runtime call failed (ctx poisoned)     */
} ofista_status;

/* Dictionaries W (the paper's H of Section III-A, N x M, real):
   IDENTITY: W = I.
   HAAR2D: orthonormal separable 2-D Haar basis, haar_levels levels, nested
     (Mallat) coefficient layout.
   EDGELET: the over-complete binary edgelets of Section III-A on a square grid
     (n = n_x = n_y).  An atom is a rotation psi (degrees, from
     edge_rotations_deg, converted with the constant pi/180), a length l in
     pixels (from edge_lengths, 1 <= l <= n-1) and an integer centre (x0, y0)
     (x = column, y = row).  Its pixels are the distinct roundings of
     (x0 + u cos psi, y0 + u sin psi), u = t - (l-1)/2, t = 0 .. l-1, each
     coordinate rounded as floor(v + 0.5 - 1e-9) (nearest, ties down); atoms
     with a pixel off the grid are dropped.  W[p, m] = 1 on the pixels of atom
     m.  Atoms are ordered by rotation, then length (as listed), then centre
     row, then centre column. */
enum { OFISTA_DICT_IDENTITY = 0, OFISTA_DICT_HAAR2D = 1, OFISTA_DICT_EDGELET = 2 };
/* Arithmetic of the Gram update: FP32 MFMA, or BF16 MFMA on a hi+lo split of
   each operand (three products, FP32 accumulation; needs n_freq divisible by
   32, else OFISTA_E_UNSUPPORTED). */
enum { OFISTA_PREC_FP32 = 0, OFISTA_PREC_SPLIT_BF16 = 1 };
/* Workgroup layout of the split-BF16 Gram update (the same sums in the same
   order, so H is bitwise the same): AUTO = BLOCK from 256 tile rows on, else
   TILE; TILE = one 64 x 64 tile per workgroup (a 32 x 32 quadrant per wave);
   BLOCK = 2 x 2 tiles per workgroup (a whole tile per wave).  Must be AUTO
   with FP32 (else OFISTA_E_UNSUPPORTED). */
enum { OFISTA_GRAM_AUTO = 0, OFISTA_GRAM_TILE = 1, OFISTA_GRAM_BLOCK = 2 };
/* How the FISTA steps of a reconstruct call run (the same iterates bit for
   bit either way):
   LAUNCHES = two kernel launches per step (the pass over the H tiles, then
     the shrink / momentum / power update);
   RESIDENT = one cooperative launch per call (up to 64 steps; more run as
     several launches), one workgroup per CU, the two phases of every step
     separated by grid barriers; each workgroup keeps its share of the H
     tiles resident (partly in LDS) across the steps.  Needs a device with
     cooperative launch, storage GRAM and at most 5 work items (runs of two
     tiles of a tile row) per CU (on 256 CUs: up to 70 tile rows, M <= 4480;
     else OFISTA_E_UNSUPPORTED at create); a reconstruct that records for
     ofista_backward uses LAUNCHES.
     If a grid barrier times out (a launch that was not co-resident), the
     results of that call are invalid and the next ofista_state returns
     OFISTA_E_HIP;
   AUTO = LAUNCHES (the faster of the two on MI355X: at M = 4096, 17.6 us
     against 26 us per step). */
enum { OFISTA_STEP_AUTO = 0, OFISTA_STEP_LAUNCHES = 1, OFISTA_STEP_RESIDENT = 2 };
/* L_n rule (Section III-B asks for L >= ||sum G^H G||_2; Section III-C bounds
   its growth by ||G_n||_2^2 per pulse):
   RUNNING = rho + the sum of sigma^2 over the pulses pushed since the last
     FISTA step (rho: Rayleigh quotient of a power vector advanced once per
     FISTA step on that step's H; 0 before any step), so several pushes
     between reconstructions each add their increment;
   BOUND = L_{n-1} + sigma_n^2 (the incremental bound taken literally).
   sigma_n^2 = ||A_s||_2^2 = lambda_max(A_s A_s^H), computed for every
   position at ofista_create in FP64 to rounding: bisection on a
   positive-definiteness test (Levinson-Durbin on the Toeplitz A_s A_s^H of
   the identity and Haar dictionaries; Householder tridiagonalisation and
   Sturm counts for the edgelet dictionary), taking the upper end. */
enum { OFISTA_LIP_RUNNING = 0, OFISTA_LIP_BOUND = 1 };
/* What the state keeps (Section III-D, Table I).  GRAM: the running sufficient
   statistics H_n, b_n (Online FISTA).  PULSES: the comparator that keeps every
   received pulse (G_k = F_k W and d_k e^{-i phase_corr}, up to max_pulses of
   them) and forms the gradient matrix-free, sum_k G_k^H (G_k z - d_k), with the
   same lambda, L rule and momentum -- the same iterates in exact arithmetic,
   different memory and work.  PULSES needs max_pulses >= 1, record_every = 0
   and FP32; ofista_gram, ofista_gram_entries, the state record and
   ofista_backward return OFISTA_E_UNSUPPORTED with it, and a push beyond
   max_pulses returns OFISTA_E_STATE. */
enum { OFISTA_STORE_GRAM = 0, OFISTA_STORE_PULSES = 1 };
/* Momentum across pulses: FISTA = t carried from pulse to pulse (Algorithm 1);
   RESTART = t = 1 at every reconstruct; ISTA = no momentum (beta = 0). */
enum { OFISTA_MOMENTUM_FISTA = 0, OFISTA_MOMENTUM_RESTART = 1, OFISTA_MOMENTUM_ISTA = 2 };

typedef struct ofista_config {
  int32_t n_x, n_y;        /* pixel grid; N = n_x*n_y >= 1                    */
  double x0, y0, dx, dy;   /* centre of pixel (0,0) and spacing, metres       */
  int32_t n_pos;           /* platform positions available to push_pulse      */
  const double *pos_xyz;   /* host, n_pos*3 doubles (x, y, z per position);
                              copied during ofista_create                     */
  int32_t n_freq;          /* K >= 1 frequencies per pulse                    */
  double freq0_hz;         /* f_0                                             */
  double dfreq_hz;         /* f_{k+1} - f_k                                   */
  int32_t dict;            /* OFISTA_DICT_*; HAAR2D needs n_x == n_y, both
                              divisible by 2^haar_levels, and N <= 8192       */
  int32_t haar_levels;     /* levels of the 2-D Haar dictionary (>= 1)        */
  double lambda;           /* l1 weight; if lambda_relative != 0 it is the
                              factor r in lambda = r * max_i |A_1^H d_1|_i,
                              fixed at the first pulse                       */
  int32_t lambda_relative;
  int32_t precision;       /* OFISTA_PREC_*                                    */
  int32_t lipschitz;       /* OFISTA_LIP_*                                     */
  int32_t momentum;        /* OFISTA_MOMENTUM_*                                */
  int32_t record_every;    /* > 0: keep what ofista_backward needs, with a
                              state checkpoint every record_every pulses
                              (see ofista_backward)                          */
  int32_t max_pulses;      /* pulses that can be recorded (record_every > 0)
                              or stored (storage = PULSES)                    */
  int32_t max_iters;       /* inner steps per reconstruct that can be
                              recorded (record_every > 0)                    */
  int32_t n_edge_lengths;  /* EDGELET: number of lengths (>= 1)               */
  const int32_t *edge_lengths;      /* host, copied during ofista_create      */
  int32_t n_edge_rotations;         /* EDGELET: number of rotations (>= 1)    */
  const double *edge_rotations_deg; /* host, degrees, copied                  */
  int32_t backprojection;  /* != 0: push_pulse also accumulates the BP image
                              (see ofista_bp_image)                          */
  int32_t storage;         /* OFISTA_STORE_*                                   */
  int32_t gram_layout;     /* OFISTA_GRAM_* (split-BF16 only)                  */
  int32_t validate_input;  /* != 0: ofista_push_pulse checks every sample of
                              d_s and returns OFISTA_E_ARG, changing nothing,
                              if one is not finite (costs a stream sync)   */
  int32_t step_kernel;     /* OFISTA_STEP_*                                    */
} ofista_config;

typedef struct ofista_stats {
  int64_t n_pulses;        /* pulses pushed since create/reset                */
  int64_t n_iters;         /* FISTA steps run since create/reset              */
  double t;                /* momentum scalar t_n                             */
  double L;                /* current L_n                                     */
  double tau;              /* 1/L_n                                           */
  double lambda;           /* l1 weight in use (0 before the first pulse when
                              relative)                                       */
  double rho;              /* Rayleigh quotient of the running power vector   */
  double sigma2;           /* ||A_s||_2^2 of the last pushed pulse            */
} ofista_stats;

/* Section III-D / Table I: the storage of Online FISTA is the sufficient
   statistics (H: the M x M Gram, kept as its packed Hermitian upper triangle,
   and b: M entries) plus the coefficients, independent of the pulse count.
   Device bytes the workspace must have for cfg (H, b, coefficient and momentum
   vectors, power vector, matvec partials, one pulse's A_s, tables, the partial
   tiles of the FP32 Gram update's split remainder (at most 255 x 8 tiles of
   32 KB, 8 MB at N = 4096), and the
   recording buffers when record_every > 0).  Pure host function, needs no GPU.
   Returns 0 when cfg is invalid. */
size_t ofista_workspace_bytes(const ofista_config *cfg);

/* Checks cfg without touching the GPU; OFISTA_OK if ofista_create would
   accept it (workspace aside). */
ofista_status ofista_check_config(const ofista_config *cfg);

/* M, the number of coefficients (dictionary atoms) for cfg; -1 when cfg is
   invalid.  Pure host function. */
int64_t ofista_coef_count(const ofista_config *cfg);

/* init(scene, geometry, lambda): the problem of Section III-B (the weighted
   LASSO over the coefficients of the dictionary of Section III-A, with the
   forward model of Section II on the given grid, positions and frequencies)
   before any pulse, H = 0 and b = 0 (Section III-C).  Validates cfg, carves the caller-owned
   workspace (device memory of at least ofista_workspace_bytes(cfg) bytes,
   256-byte aligned, kept alive by the caller until ofista_destroy), copies the
   host tables, precomputes ||A_s||_2^2 for every position (it depends only on
   the geometry; for EDGELET by forming A_s A_s^H per position in FP64, using
   the H region of the workspace as scratch, OFISTA_E_UNSUPPORTED if
   K*K*16 bytes exceed that region) and zeroes the state.  hip_stream is a hipStream_t (NULL =
   the null stream).  The ctx (host memory) is owned by the library. */
ofista_status ofista_create(const ofista_config *cfg, void *d_workspace,
                            size_t workspace_bytes, void *hip_stream,
                            struct ofista_ctx **out);

/* Zero the online state (H, b, c, t, L, lambda, power vector, pulse count) --
   the start of the Section III-C recursions, H_0 = 0 and b_0 = 0 -- so that a
   new image can be formed with the same geometry tables. */
ofista_status ofista_reset(struct ofista_ctx *ctx);

/* push_pulse(d_s, s): one received pulse, Section III-C: the Delta-A / Delta-b
   equations (H += A_s^H A_s, b += A_s^H d_s with R_n = I) folded into the
   A_n / b_n recursions, and the step bound grown by ||A_s||_2^2 (the
   incremental bound; see OFISTA_LIP_*).  d_pulse: device, K complex64; s:
   index of the platform position (0 <= s < n_pos; positions may repeat or be
   skipped).  The data used is d_s * exp(-i phase_corr).  Enqueues A_s, the H
   and b updates, lambda at the first pulse, and L_n, tau. */
ofista_status ofista_push_pulse(struct ofista_ctx *ctx, const void *d_pulse,
                                int32_t s, double phase_corr);

/* reconstruct(iters): Algorithm 1 with iters inner steps on the current
   (H_n, b_n), warm-started from c_hat_{n-1} and t_{n-1}.  iters may be 0.
   d_coef_out: device, M complex64, receives c_hat_n (NULL = not copied).
   OFISTA_E_STATE before the first pulse. */
ofista_status ofista_reconstruct(struct ofista_ctx *ctx, int32_t iters,
                                 void *d_coef_out);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same
   as ofista_reconstruct -- same kernels, same order, bitwise the same result
   -- but the FISTA step's matvec partials (nb x nb x 64 x 16 bytes, nb =
   ceil(M / 64)) live in a fixed 16 MiB array in device memory that the library
   holds on every GPU it runs on until the process ends, instead of in the
   ctx's workspace.  Nothing in that array needs to start at zero (every step
   reads only the partials it wrote).  Allocates nothing: no hipMalloc,
   hipFree, event creation or host allocation (profiling events are not taken
   in this call).  Every ctx on one GPU shares the array, so calls that
   overlap on one GPU (different streams or threads) race and must be
   serialised by the caller.  OFISTA_E_UNSUPPORTED when the partials exceed
   the array (M > 8192) or with PULSES storage; otherwise the statuses of
   ofista_reconstruct. */
ofista_status ofista_reconstruct_static(struct ofista_ctx *ctx, int32_t iters,
                                        void *d_coef_out);

/* Image x = W c_hat (Section III-B, rho ~ H c with the paper's dictionary H).
   d_img_out: device, N complex64. */
ofista_status ofista_image(struct ofista_ctx *ctx, void *d_img_out);

/* BP baseline of Section IV-A: d_img_out (device, N complex64) receives
   (1/n) sum over the n pushed pulses of F_s^H (d_s e^{-i phase_corr}), the
   adjoint-imaged pulses averaged in the pixel domain (display it as
   20 log10 |.|).  Needs backprojection != 0 in the config (else
   OFISTA_E_STATE), and n >= 1 (else OFISTA_E_STATE).  The accumulator is
   part of the state record. */
ofista_status ofista_bp_image(struct ofista_ctx *ctx, void *d_img_out);

/* Large-coefficient count of Section IV-B: the number of entries of c_hat
   with |c| > threshold, |c| formed in FP32 (sqrtf of the FP32 sum of
   squares) and compared with (float)threshold.  Synchronises the stream
   (the count is returned on the host). */
ofista_status ofista_count_large(struct ofista_ctx *ctx, double threshold, int64_t *count);

/* Host copy of the scalar state: the pulse and step counts, the momentum
   scalar t of Algorithm 1, L_n and tau = 1/L_n (Section III-B), lambda, and
   the running spectral estimate.  Synchronises the stream. */
ofista_status ofista_state(struct ofista_ctx *ctx, ofista_stats *out);

/* Synthetic radar return for position s (the Section II measurement model):
   d = exp(i phase_err) F_s rho + sigma * noise, sigma^2 = |F_s rho|^2 / K *
   10^(-snr_db/10).  d_rho: device, N complex64 pixel reflectivities; d_noise:
   device, K complex64 unit-variance draws, or NULL for a noiseless echo;
   d_out: device, K complex64.  Uses the ctx's scratch rows (do not overlap
   with push_pulse on another thread -- ctx calls never overlap anyway). */
ofista_status ofista_echo(struct ofista_ctx *ctx, int32_t s, const void *d_rho,
                          const void *d_noise, double snr_db, double phase_err,
                          void *d_out);

/* Inspection.  ofista_rows: A_s for position s into d_out (K x M complex64,
   row k contiguous).  ofista_gram: the Hermitian H_n expanded to a dense
   M x M complex64 matrix (row-major; M <= 16384, else OFISTA_E_UNSUPPORTED).
   ofista_vector: which = 0 b, 1 c_hat, 2 power vector w (unnormalised), M
   complex64 each. */
ofista_status ofista_rows(struct ofista_ctx *ctx, int32_t s, void *d_out);
/* Sampled entries out[t] = H_n[i[t], j[t]] for t < n, read from the packed
   storage at any M.  d_i, d_j: device int32 arrays of n coefficient indices;
   d_out: device, n complex64.  Indices outside [0, M) give NaN. */
ofista_status ofista_gram_entries(struct ofista_ctx *ctx, int32_t n, const int32_t *d_i,
                                  const int32_t *d_j, void *d_out);
ofista_status ofista_gram(struct ofista_ctx *ctx, void *d_out);
ofista_status ofista_vector(struct ofista_ctx *ctx, int32_t which, void *d_out);

/* Resumable state record: the sufficient statistics of Section III-C (H_n and
   b_n carry everything the past pulses contribute, so resuming from them
   equals the uninterrupted run) plus the iteration state of Algorithm 1
   (n, t, L, lambda, power vector, c_hat) and the BP accumulator when
   enabled.  The
   buffer is caller-owned device memory of ofista_state_bytes(cfg) bytes;
   alignment padding inside it is left unwritten.  Export synchronises the
   stream; import synchronises it and forgets any recorded history. */
size_t ofista_state_bytes(const ofista_config *cfg);  /* 0 for PULSES storage */
ofista_status ofista_export_state(struct ofista_ctx *ctx, void *d_buf);
ofista_status ofista_import_state(struct ofista_ctx *ctx, const void *d_buf);

/* Differentiation form (Section III-C run as an unrolled, differentiable map).
   With record_every > 0 in the config, every pushed pulse (data, position,
   phase_corr) and the step count of the reconstruct that follows it are
   recorded, with a state checkpoint every record_every pulses (at most
   max_pulses pulses, at most max_iters steps per reconstruct, exactly one
   reconstruct per pulse; otherwise OFISTA_E_STATE / OFISTA_E_ARG).

   ofista_backward: given d_grad_img (device, N complex64) = dLoss/dRe x +
   i dLoss/dIm x for the current image x = W c_hat of a real loss, returns
   *grad_lambda = dLoss/dlambda (lambda as an absolute value, see
   ofista_set_lambda) and grad_phase[n] = dLoss/dphase_corr_n for every pulse
   pushed since the last reset (host array of n_pulses doubles).  H, L_n and
   the momentum sequence do not depend on these parameters; the reverse pass
   re-runs each segment from its checkpoint (bitwise the same forward) and
   walks its pulses and steps backwards.  Synchronises the stream; the online
   state after the call is the state before it.  OFISTA_E_STATE when not
   recording or nothing was pushed. */
ofista_status ofista_backward(struct ofista_ctx *ctx, const void *d_grad_img,
                              double *grad_lambda, double *grad_phase);

/* Use the absolute l1 weight lambda from now on (lambda_relative is turned
   off).  Takes effect for the next FISTA step. */
ofista_status ofista_set_lambda(struct ofista_ctx *ctx, double lambda);

/* Per-kernel timing with HIP events on the ctx's stream.  While enabled, every
   launch of the named kernel class is bracketed by a pair of events.
   ofista_kernel_time synchronises and returns the summed milliseconds and the
   launch count since enabling.  kernel: 0 Gram update (with the correlation
   b += A_s^H d fused in; when the library splits the last tiles into
   frequency pieces, the pair of events spans the Gram launch and the launch
   that adds the pieces to H), 1 FISTA-step tile pass (the H z / H w streaming),
   2 rows, 3 correlation (separate launch on the split-BF16 path only),
   4 scalars (their own launch only where the FP32 Gram update has no
   fix-up launch; otherwise they run as one more workgroup of it and are
   timed with class 0), 5 FISTA-step update (slot sums, shrink, momentum, power
   vector), 6 and 7 the two passes over the stored pulses of the PULSES
   storage (G z - d, G w; then G^H of both), 8 the resident step kernel (one
   launch per reconstruct call runs all its steps, tile passes and updates;
   classes 1 and 5 then stay empty). */
ofista_status ofista_profile(struct ofista_ctx *ctx, int32_t enable);
ofista_status ofista_kernel_time(struct ofista_ctx *ctx, int32_t kernel,
                                 double *total_ms, int64_t *launches);

/* Free the host ctx (the workspace stays the caller's). NULL is ignored. */
void ofista_destroy(struct ofista_ctx *ctx);

/* Static message for a status; with a ctx, the last detailed message. */
const char *ofista_error_string(const struct ofista_ctx *ctx, ofista_status st);

/* Layout constants of the library (for tests): tile edge of the packed
   Hermitian storage. */
int32_t ofista_tile(void);

#ifdef __cplusplus
}
#endif
#endif /* OFISTA_H */
