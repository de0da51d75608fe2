// Reverse pass of the differentiation form: gradients of a real loss of the
// final image to lambda and to the per-pulse phase corrections, through the
// unrolled online run.  Only b_n and the shrink threshold alpha = lambda tau_n
// depend on the parameters, so per pulse (Algorithm 1 run backwards, complex
// adjoints xbar = dL/dRe x + i dL/dIm x):
//
//   cbar_k = P_k + (1 + beta_k) zbar_{k+1}        (P_k: partial from step k+1)
//   ubar_k = J_S(u_k)^T cbar_k                    (|u| > alpha: radial part x1,
//                                                  tangential x(1 - alpha/|u|); else 0)
//   alphabar += -Re(conj(cbar_k) u_k/|u_k|)       (active entries)
//   P_{k-1} = -beta_k zbar_{k+1}
//   zbar_k = ubar_k - tau H_n ubar_k,  bbar_n += tau ubar_k
//   c_hat_bar_{n-1} = P_0 + zbar_1,    lambdabar += tau_n alphabar
//   B += bbar_n,  dL/dphi_n = Im(sum_i conj(B_i) Delta b_n,i)
//
// H_n ubar reuses the forward tile pass (same packed tiles and slots);
// k_adj_update sums the slots and fuses the step-k and step-(k-1) elementwise
// work.  All sums are fixed-order, so gradients are bitwise reproducible.
#include "ofista_internal.h"

namespace ofista {
namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ubar = J_S(u)^T cbar for the complex soft threshold; returns the alpha
// contribution -Re(conj(cbar) uhat) (0 if inactive).
__device__ __forceinline__ float2 shrink_vjp(float2 u, float2 cb, float alpha, double *abar) {
  const float mag = sqrtf(u.x * u.x + u.y * u.y);
  if (!(mag > alpha)) {
    *abar = 0.0;
    return make_float2(0.f, 0.f);
  }
  const float hx = u.x / mag, hy = u.y / mag;
  const float p = cb.x * hx + cb.y * hy;
  const float f = 1.f - alpha / mag;
  *abar = -static_cast<double>(p);
  return make_float2(p * hx + f * (cb.x - p * hx), p * hy + f * (cb.y - p * hy));
}

// Step m of a pulse: ubar_m from the incoming c_hat_bar, P_{m-1} = 0, bbar = 0.
__global__ __launch_bounds__(64) void k_adj_start(AdjArgs a) {
  const int R = blockIdx.x;
  const int i = R * kTile + threadIdx.x;
  double ab = 0.0;
  float2 ub = make_float2(0.f, 0.f);
  if (i < a.N) ub = shrink_vjp(a.u_prev[i], a.chat_bar[i], static_cast<float>(a.scal->alpha), &ab);
  a.ubar_next[i] = ub;
  a.cpart_next[i] = make_float2(0.f, 0.f);
  a.bbar[i] = make_float2(0.f, 0.f);
  ab = wave_sum_d(ab);
  if (threadIdx.x == 0) a.alpha_parts[R] = ab;
}

constexpr int kAdjBatch = 16;

// Step k: y = H ubar_k from the slots; zbar_k, bbar; then step k-1's ubar and
// partial, or (k = 1) the adjoint of the previous pulse's coefficients.
__global__ __launch_bounds__(256) void k_adj_update(AdjArgs a) {
  __shared__ float2 red[256];
  const int R = blockIdx.x;
  const int nb = a.nb;
  const int t = threadIdx.x;
  const int r = t & 63, part = t >> 6;
  float2 acc = make_float2(0.f, 0.f);
  const float4 *q = a.Q + r;
  for (int j0 = part; j0 < nb; j0 += 4 * kAdjBatch) {
    float4 v[kAdjBatch];
#pragma unroll
    for (int u = 0; u < kAdjBatch; ++u) {
      const int j = j0 + 4 * u;
      v[u] = q[slot_index(j < nb ? j : nb - 1, R, nb) * kTile];
    }
#pragma unroll
    for (int u = 0; u < kAdjBatch; ++u) {
      const int j = j0 + 4 * u;
      const bool ok = j < nb && (j < R || ((j - R) % a.chunk) == 0);
      acc.x += ok ? v[u].x : 0.f;
      acc.y += ok ? v[u].y : 0.f;
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t >= 64) return;
  float2 y = red[t];
#pragma unroll
  for (int p = 1; p < 4; ++p) {
    y.x += red[t + 64 * p].x;
    y.y += red[t + 64 * p].y;
  }
  const int i = R * kTile + t;
  const float tau = static_cast<float>(a.scal->tau);
  const float alpha = static_cast<float>(a.scal->alpha);
  double ab = 0.0;
  if (i < a.N) {
    const float2 ub = a.ubar_cur[i];
    const float2 zb = make_float2(ub.x - tau * y.x, ub.y - tau * y.y);
    float2 bb = a.bbar[i];
    bb.x += tau * ub.x;
    bb.y += tau * ub.y;
    a.bbar[i] = bb;
    const float2 cp = a.cpart_cur[i];
    if (a.last) {
      a.chat_bar[i] = make_float2(cp.x + zb.x, cp.y + zb.y);
    } else {
      const float2 cb = make_float2(cp.x + (1.f + a.beta_prev) * zb.x, cp.y + (1.f + a.beta_prev) * zb.y);
      a.ubar_next[i] = shrink_vjp(a.u_prev[i], cb, alpha, &ab);
      a.cpart_next[i] = make_float2(-a.beta_prev * zb.x, -a.beta_prev * zb.y);
    }
  } else if (!a.last) {
    a.ubar_next[i] = make_float2(0.f, 0.f);
    a.cpart_next[i] = make_float2(0.f, 0.f);
  }
  if (!a.last) {
    ab = wave_sum_d(ab);
    if (t == 0) a.alpha_parts[R] = ab;
  }
}

// End of a pulse: lambdabar_n = tau_n sum(alpha parts), B += bbar_n,
// dL/dphi_n = Im(sum conj(B) Delta b_n).  One workgroup, fixed-order sums.
__global__ __launch_bounds__(256) void k_adj_pulse(const AdjArgs a, int n_parts, int Npad,
                                                   const float2 *__restrict__ dB,
                                                   double *__restrict__ lam_out,
                                                   double *__restrict__ phase_out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < n_parts; j += 256) s += a.alpha_parts_all[j];
  double ph = 0.0;
  for (int i = threadIdx.x; i < Npad; i += 256) {
    float2 B = a.Bbar[i];
    const float2 bb = a.bbar[i];
    B.x += bb.x;
    B.y += bb.y;
    a.Bbar[i] = B;
    const float2 d = dB[i];
    // Im(conj(B) d) = B.x d.y - B.y d.x
    ph += static_cast<double>(B.x) * d.y - static_cast<double>(B.y) * d.x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double stot = red[0];
  __syncthreads();
  red[threadIdx.x] = ph;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *lam_out = a.scal->tau * stot;
    *phase_out = red[0];
  }
}

__global__ void k_set_lambda(DevScalars *scal, double lam) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal->lam = lam;
    scal->alpha = lam * scal->tau;
  }
}

}  // namespace

hipError_t launch_adj_start(const AdjArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_start, dim3(a.nb), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adj_update(const AdjArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_update, dim3(a.nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adj_pulse(const AdjArgs &a, int n_parts, int Npad, const float2 *dB,
                            double *lam_out, double *phase_out, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_pulse, dim3(1), dim3(256), 0, st, a, n_parts, Npad, dB, lam_out,
                     phase_out);
  return hipGetLastError();
}

hipError_t launch_set_lambda(DevScalars *scal, double lam, hipStream_t st) {
  hipLaunchKernelGGL(k_set_lambda, dim3(1), dim3(64), 0, st, scal, lam);
  return hipGetLastError();
}

}  // namespace ofista
