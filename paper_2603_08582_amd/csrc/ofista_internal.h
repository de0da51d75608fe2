// Internal declarations of libofista: device-side layout constants, the
// device scalar block, and the kernel launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>

#include "host_plan.h"

namespace ofista {

static_assert(sizeof(float2) == kBytesC64 && sizeof(float4) == kBytesF4 &&
                  sizeof(double2) == kBytesD2 && sizeof(int2) == kBytesI2,
              "layout byte sizes");

// Vector types for nontemporal loads (the builtin takes scalar or
// ext_vector_type pointers only).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Slot of the matvec partials (nb x nb slots of kTile float4) that holds the
// contribution of source tile row/column v to target tile row R.  Row partials
// (v >= R, the run start of tile row R) sit at [R][v], the upper part
// including the diagonal.  Column partials (v < R, from tile (v, R)) sit at
// [nb-1-v][nb-1-R], strictly below the diagonal, so the column partials one
// work item writes are adjacent and those of one source row are contiguous.
__host__ __device__ inline size_t slot_index(int v, int R, int nb) {
  return v >= R ? static_cast<size_t>(R) * nb + v
                : static_cast<size_t>(nb - 1 - v) * nb + (nb - 1 - R);
}
constexpr double kC0 = 299792458.0;  // speed of light, m/s
constexpr double kPi = 3.141592653589793238462643383279502884;

// Geometry passed by value.  N is the coefficient count M (the length of b,
// c and every FISTA vector; Npad = M rounded up to kTile), npix = nx*ny the
// pixel count (N == npix except for the edgelet dictionary).
struct Geom {
  int nx, ny, N, Npad, K, npos, npix;
  double x0, y0, dx, dy;
  double f0, df;
};

// Dictionary of the forward rows and the image.  Edgelet atoms are stored
// twice as compressed index lists: atom -> pixels and pixel -> atoms (both in
// increasing order), so that A = F W and x = W c are gathers with a fixed
// summation order.
struct DictTabs {
  int kind;              // OFISTA_DICT_* value
  int levels;            // Haar levels
  const int *atom_ptr;   // M + 1 offsets into atom_pix
  const int *atom_pix;
  const int *pix_ptr;    // npix + 1 offsets into pix_atom
  const int *pix_atom;
};

// Device-side pointers of one context, carved from the workspace.
struct DevState {
  float2 *H;         // packed tiles
  float2 *A;         // K x Npad rows of the current pulse (scratch)
  float2 *b;
  float2 *cbuf[2];   // c_hat, ping-pong by step parity
  float2 *zbuf[2];   // momentum point z
  float2 *wbuf[2];   // power vector
  float4 *Q;         // matvec partials, nb x nb x kTile of (yz, yw)
  double *slots[2];  // per update workgroup: [0, P) Re<w, Hw> parts, [P, 2P) |w'|^2 parts, P = nparts
  DevScalars *scal;
  double *pos;       // npos x 3
  double *sig2;      // npos, ||A_s||_2^2 per position
  double2 *gtoep;    // npos x K, Toeplitz generator of A_s A_s^H
  int2 *tile_ij;     // logical tile -> (I, J), padded to a multiple of 8
  int *tile_row0;    // index of tile (I, I)
  WorkItem *items;
  int *atom_ptr, *atom_pix, *pix_ptr, *pix_atom;  // edgelet tables (else NULL)
  float2 *bp;        // BP accumulator, npix (NULL when not enabled)
  unsigned *counter; // one word for ofista_count_large
  unsigned *bar;     // 8 grid-barrier counters, kBarStride apart
  double2 *echo_tmp; // K clean-echo sums
  // split-BF16 operands of the Gram update, Npad x K words (NULL for FP32)
  unsigned *Ahi;
  unsigned *Alo;
};

// ---- rows.hip ----
hipError_t launch_rows(const Geom &g, const double *pos, int s, float2 *A,
                       const DictTabs &dt, hipStream_t st);
// x = W c (npix entries).
hipError_t launch_image(const Geom &g, const float2 *c, float2 *x, const DictTabs &dt,
                        hipStream_t st);
// c = W^T x (adjoint of the image synthesis), padded to Npad.
hipError_t launch_image_adjoint(const Geom &g, const float2 *x, float2 *c, const DictTabs &dt,
                                hipStream_t st);
// bp[p] += sum_k conj(F_s[k, p]) d_k e^{-i phi} for every pixel p.
hipError_t launch_backproject(const Geom &g, const double *pos, int s, const float2 *d,
                              double cos_c, double sin_c, float2 *bp, hipStream_t st);
hipError_t launch_echo(const Geom &g, const double *pos, int s,
                       const float2 *rho, const float2 *noise, double snr_db,
                       double phase_err, double2 *tmp, float2 *out,
                       hipStream_t st);
// sigma^2 = ||A_s||_2^2 for every position (identity and Haar dictionaries,
// where A_s A_s^H is Hermitian Toeplitz): FP64 generator, then bisection with
// a Levinson-Durbin definiteness test.
hipError_t launch_sigma2(const Geom &g, const double *pos, double2 *gtoep,
                         double *sig2, hipStream_t st);
// Dense route to sigma^2 (any dictionary): G = A A^H (K x K, FP64 sums) from
// the K x Npad rows A, then the largest eigenvalue of nmat such matrices
// stored back to back (FP64 Householder tridiagonalisation in place -- the
// matrices are destroyed -- and Sturm bisection), one workgroup each, results
// to sig2[0 .. nmat).
hipError_t launch_gram_kk(const Geom &g, const float2 *A, double2 *G, hipStream_t st);
hipError_t launch_sigma2_dense(int K, double2 *G, int nmat, double *sig2, hipStream_t st);

// ---- gram.hip ----
// Correlation as its own launch (split-BF16 path): b += A^H (d e^{-i phi}).
// With b == NULL only Delta b is written (to delta, if set).
hipError_t launch_corr(const Geom &g, const float2 *A, const float2 *d,
                       double cos_c, double sin_c, float2 *b, DevScalars *scal,
                       int first, hipStream_t st, float2 *delta = nullptr);
// Split-BF16 Gram update (K must be a multiple of 32): split A into the
// pixel-major hi/lo planes, then H += A^H A from three BF16 products.
// Launchers of the timed kernels take optional events (t0, t1): when given,
// they bracket that one kernel's execution (hipExtLaunchKernelGGL).
// With blocks (nblocks 2 x 2 tile blocks (IB, JB), IB <= JB) the product runs
// one 64 x 64 tile per wave over those blocks (same sums, fewer LDS reads per
// MFMA, used for large N); otherwise one tile per workgroup over tile_ij.
hipError_t launch_gram_bf16x3(const Geom &g, const float2 *A, unsigned *Ahi, unsigned *Alo,
                              float2 *H, const int2 *tile_ij, int ntiles_grid, const int2 *blocks,
                              int nblocks, hipStream_t st, hipEvent_t t0 = nullptr,
                              hipEvent_t t1 = nullptr);
// Correlation fused into the Gram update: b += A^H (d e^{-i phi}).
struct CorrArgs {
  const float2 *d;
  float cphi, sphi;
  float2 *b;
  DevScalars *scal;
  int first;  // also record max |Delta b| (first pulse)
};
// Remainder split of the FP32 Gram update.  When the tile count is a few
// rounds of one tile per CU plus a remainder, the last off-diagonal tiles are
// split along the frequencies into `parts` pieces that run after the whole
// tiles; each piece writes its 64 x 64 partial to P (tile-major, row-major
// inside), and a second launch adds the pieces of each split tile in
// increasing order and then adds that sum to H.  Table entries: x = I | split
// index << 16, y = J | piece << 20 (piece 0: whole tile, 1..parts: part).
struct GramSplit {
  float2 *P;        // nsplit * parts partial tiles
  const int2 *ij;   // (I, J) of each split tile
  int nsplit, parts;
};
struct ScalarArgs;
// With sc given and the split on, the fix-up launch also runs the pulse
// scalars (one more workgroup) and *sc_done is set; otherwise *sc_done is
// cleared and the caller launches them.
hipError_t launch_gram_fp32(const Geom &g, const float2 *A, float2 *H,
                            const int2 *tile_ij, int ntiles_grid, const CorrArgs &corr,
                            const GramSplit &split, int kb, const ScalarArgs *sc, bool *sc_done,
                            hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_gram_entries(const Geom &g, const float2 *H, const int *tile_row0, int n,
                               const int *ii, const int *jj, float2 *out, hipStream_t st);
hipError_t launch_gram_dense(const Geom &g, const float2 *H,
                             const int *tile_row0, float2 *out,
                             hipStream_t st);

// ---- fista.hip ----
struct StepArgs {
  const float2 *H;
  const float2 *zc;
  const float2 *wc;
  const float2 *b;
  const float2 *cc;
  float2 *cn;
  float2 *zn;
  float2 *wn;
  float4 *Q;
  const double *slot_prev;
  double *slot_cur;
  const DevScalars *scal;
  const WorkItem *items;
  float2 *urec;  // if set, the update stores u = z - tau (H z - b) here
  int nb, N, nitems, chunk;
  int h_cached;  // tile pass: cached (H fits the last-level cache) or nontemporal H loads
  int slot_nt;   // tile pass: nontemporal slot stores (the slots exceed the last-level cache)
  float beta;
  // store-all comparator: the update sums nchunks partial rows of P (stride
  // Npad) instead of the tile-pass slots
  const float4 *P;
  int nchunks, Npad;
};
// All FISTA steps of one reconstruct call in one cooperative launch (one
// workgroup per CU, grid barriers between the phases of a step); see
// k_steps_resident.
constexpr int kResMaxSteps = 64;   // steps per launch
constexpr int kResLdsItems = 2;    // work items per workgroup whose tiles stay in LDS
constexpr int kResRegItems = 2;    // work items per workgroup whose tiles stay in registers
constexpr int kResMaxItems = 5;    // work items per workgroup (z, w staged in LDS per item)
constexpr int kResMaxParts = 1024; // update parts kUpdSplit * nb (summed per thread in registers)
struct ResidentArgs {
  const float2 *H;
  const WorkItem *items;
  const float2 *b;
  float2 *zbuf[2], *cbuf[2], *wbuf[2];
  double *slots[2];
  float4 *Q;
  DevScalars *scal;
  unsigned *bar;       // 8 arrival counters, kBarStride apart
  unsigned bar_gen;    // barriers completed on the counters before this launch
  int nb, N, nitems, nparts;
  int p0;              // buffer parity of the first step
  int iters;           // steps of this launch (<= kResMaxSteps)
  int warm;            // != 0: the first step multiplies c (z^(1) = c_{n-1})
  float beta[kResMaxSteps];
};
hipError_t launch_steps_resident(const ResidentArgs &a, int nwg, hipStream_t st);
// Workgroups the resident step kernel needs resident at once (one per CU),
// or 0 when the device cannot run it (no cooperative launch, or too few
// resources per CU).
int resident_grid(int device, int n_cu);
hipError_t launch_step_tiles(const StepArgs &a, hipStream_t st, hipEvent_t t0 = nullptr,
                             hipEvent_t t1 = nullptr);
hipError_t launch_step_update(const StepArgs &a, hipStream_t st, hipEvent_t t0 = nullptr,
                              hipEvent_t t1 = nullptr);
// Store-all comparator.  U[r] = (G_r z - D_r, G_r w) for the rows r < rows of
// the stacked operator (rows x Npad, M used); P[c][m] = sum over rows
// r in [64c, 64c + 64) of conj(G[r, m]) U[r]; then launch_step_update with
// P set.  D: rows complex64 (the rotated data).
hipError_t launch_store_forward(const float2 *G, const float2 *D, int rows, int Npad, int M,
                                const float2 *z, const float2 *w, float4 *U, hipStream_t st,
                                hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_store_adjoint(const float2 *G, int rows, int Npad, const float4 *U, float4 *P,
                                hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// out[k] = d[k] e^{-i phi}, k < K.
hipError_t launch_rotate(const float2 *d, int K, double cos_c, double sin_c, float2 *out,
                         hipStream_t st);
// Per-pulse scalars: lambda (first pulse), sigma^2 of position s, L_n, tau,
// alpha.  L_n (RUNNING) = rho + the sigma^2 of every pulse pushed since the
// last FISTA step (Weyl: lambda_max(H + sum dH) <= lambda_max(H) + sum
// ||dH||_2), rho the Rayleigh quotient of that step's power vector, formed
// from its slots when steps ran since the previous push (new_rho) and kept
// from then on otherwise.  BOUND: L_{n-1} + sigma_n^2.
struct ScalarArgs {
  DevScalars *scal;
  const double *sig2;
  const double *slot_r, *slot_m;  // Re<w, Hw> and |w|^2 parts of the last step
  double lam_in;
  int s, first, rel, lip, new_rho, nparts;
};

// The scalars as one 256-thread workgroup (its own launch, or an extra
// workgroup of the Gram fix-up launch); the slot sums use a fixed-order tree,
// so both places give the same bits.
__device__ inline double scalars_tree_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
__device__ inline void pulse_scalars(const ScalarArgs &a, double *red) {
  DevScalars *scal = a.scal;
  // every value from memory is read before the reductions, so they arrive
  // in one round trip rather than one after another
  const double sigma2 = a.sig2[a.s];
  const double rho_kept = scal->rho, acc_kept = scal->sig2_acc, L_prev = scal->L;
  const double lam_kept = scal->lam;
  const unsigned dbmax_bits = scal->dbmax_bits;
  double rho = 0.0;
  if (a.new_rho) {
    double pr = 0.0, pm = 0.0;
    for (int j = threadIdx.x; j < a.nparts; j += 256) {
      pr += a.slot_r[j];
      pm += a.slot_m[a.nparts + j];
    }
    const double rs = scalars_tree_sum(pr, red);
    const double ms = scalars_tree_sum(pm, red);
    rho = rs / ms;
  }
  if (threadIdx.x != 0) return;
  const double lam =
      a.first ? (a.rel ? a.lam_in * static_cast<double>(__uint_as_float(dbmax_bits)) : a.lam_in)
              : lam_kept;
  double acc = sigma2;
  if (a.new_rho) {
    scal->rho = rho;
  } else {
    rho = rho_kept;
    acc += acc_kept;
  }
  const double L = a.lip == 0 ? rho + acc : L_prev + sigma2;
  scal->lam = lam;
  scal->sig2_acc = acc;
  scal->sigma2 = sigma2;
  scal->L = L;
  scal->tau = 1.0 / L;
  scal->alpha = lam / L;
}

hipError_t launch_scalars(const ScalarArgs &a, hipStream_t st);
hipError_t launch_fill(void *p, size_t n_u32, unsigned value, hipStream_t st);
// *count (zeroed by the caller) += #{m < M : |c_m| > thr} (FP32 magnitude).
hipError_t launch_count_large(const float2 *c, int M, float thr, unsigned *count, hipStream_t st);
// *count = number of the K samples of d with a non-finite component.
hipError_t launch_count_nonfinite(const float2 *d, int K, unsigned *count, hipStream_t st);
// out[i] = x[i] * scale for i < n.
hipError_t launch_scale(const float2 *x, float scale, int n, float2 *out, hipStream_t st);
hipError_t launch_init_power(float2 *w, double *slot0, double *slot1, int N,
                             int Npad, int nb, hipStream_t st);

// ---- adjoint.hip ----
struct AdjArgs {
  const float4 *Q;
  const DevScalars *scal;          // tau_n, alpha_n of the pulse being reversed
  const float2 *u_prev;            // u of the step whose ubar is formed
  const float2 *ubar_cur;          // ubar_k (input of the update)
  float2 *ubar_next;               // ubar of the next reverse step
  const float2 *cpart_cur;         // partial adjoint P_{k-1}
  float2 *cpart_next;              // P_{k-2}
  float2 *bbar;                    // adjoint of b_n (this pulse)
  float2 *chat_bar;                // adjoint of the coefficients entering / leaving the pulse
  float2 *Bbar;                    // sum of bbar over later pulses
  double *alpha_parts;             // nb parts of alphabar for the step whose ubar is formed
  const double *alpha_parts_all;   // all parts of the pulse (k_adj_pulse)
  int nb, N, chunk, last;
  float beta_prev;
};
hipError_t launch_adj_start(const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_update(const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_pulse(const AdjArgs &a, int n_parts, int Npad, const float2 *dB,
                            double *lam_out, double *phase_out, hipStream_t st);
hipError_t launch_set_lambda(DevScalars *scal, double lam, hipStream_t st);

}  // namespace ofista
