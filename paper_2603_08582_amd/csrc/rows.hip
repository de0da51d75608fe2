// Forward-operator rows, dictionary fold, image synthesis, synthetic echo and
// the per-position spectral norm ||A_s||_2^2.
//
// The kernel of F_s (Section II: amplitude 1, phase t - 2|gamma(s) - x|/c on a
// stepped-frequency grid) is exp(-i 4 pi f_k R / c0).  At X band and 10 km the
// phase is ~4e6 rad, where an FP32 ulp is 0.5 rad, so range and phase are
// formed in FP64 and reduced modulo 2 pi in FP64 (two-constant Cody-Waite
// split of 2 pi) before the FP32 sine/cosine.
#include "ofista_internal.h"

namespace ofista {
namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;
constexpr double k2PiHi = 6.283185307179586232;   // fl(2 pi)
constexpr double k2PiLo = 2.4492935982947064e-16;  // 2 pi - fl(2 pi)

__device__ __forceinline__ float2 phasor_neg(double phase) {
  // exp(-i phase)
  const double n = rint(phase * kInv2Pi);
  double r = fma(-n, k2PiHi, phase);
  r = fma(-n, k2PiLo, r);
  float s, c;
  sincosf(static_cast<float>(r), &s, &c);
  return make_float2(c, -s);
}

__device__ __forceinline__ double pixel_range(const Geom &g, const double *p,
                                              int i) {
  const int ix = i % g.nx;
  const int iy = i / g.nx;
  const double ex = p[0] - (g.x0 + ix * g.dx);
  const double ey = p[1] - (g.y0 + iy * g.dy);
  const double ez = p[2];
  return sqrt(ex * ex + ey * ey + ez * ez);
}

constexpr int kRowsKCh = 16;  // frequencies per thread in the identity rows

// A_s = F_s for the identity dictionary: thread per pixel, kRowsKCh
// frequencies per thread (the FP64 range is formed once per pixel).
__global__ __launch_bounds__(256) void k_rows_identity(Geom g,
                                                       const double *__restrict__ pos,
                                                       int s,
                                                       float2 *__restrict__ A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int k0 = blockIdx.y * kRowsKCh;
  if (i >= g.Npad) return;
  const int kn = min(kRowsKCh, g.K - k0);
  float2 *out = A + static_cast<size_t>(k0) * g.Npad + i;
  if (i >= g.N) {
    for (int kk = 0; kk < kn; ++kk) out[static_cast<size_t>(kk) * g.Npad] = make_float2(0.f, 0.f);
    return;
  }
  const double R = pixel_range(g, pos + 3 * s, i);
  const double c4 = 4.0 * kPi / kC0;
  for (int kk = 0; kk < kn; ++kk) {
    const double f = g.f0 + (k0 + kk) * g.df;
    out[static_cast<size_t>(kk) * g.Npad] = phasor_neg((c4 * f) * R);
  }
}

// One level of the orthonormal 2-D Haar analysis on the top-left m x m block
// of an n-wide row-major image held in LDS, in place.  Each 2 x 2 input block
// (a b / c d) produces  LL = (a+b+c+d)/2 at (y, x),  (a-b+c-d)/2 at (y, x+h),
// (a+b-c-d)/2 at (y+h, x),  (a-b-c+d)/2 at (y+h, x+h),  h = m/2.
template <int kMaxPer>
__device__ void haar_level_analysis(float2 *buf, int n, int m) {
  const int h = m >> 1;
  const int nblk = h * h;
  float2 o[kMaxPer][4];
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q >= nblk) break;
    const int y = q / h, x = q % h;
    const float2 a = buf[(2 * y) * n + 2 * x];
    const float2 b = buf[(2 * y) * n + 2 * x + 1];
    const float2 c = buf[(2 * y + 1) * n + 2 * x];
    const float2 d = buf[(2 * y + 1) * n + 2 * x + 1];
    o[u][0] = make_float2(0.5f * ((a.x + b.x) + (c.x + d.x)), 0.5f * ((a.y + b.y) + (c.y + d.y)));
    o[u][1] = make_float2(0.5f * ((a.x - b.x) + (c.x - d.x)), 0.5f * ((a.y - b.y) + (c.y - d.y)));
    o[u][2] = make_float2(0.5f * ((a.x + b.x) - (c.x + d.x)), 0.5f * ((a.y + b.y) - (c.y + d.y)));
    o[u][3] = make_float2(0.5f * ((a.x - b.x) - (c.x - d.x)), 0.5f * ((a.y - b.y) - (c.y - d.y)));
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q >= nblk) break;
    const int y = q / h, x = q % h;
    buf[y * n + x] = o[u][0];
    buf[y * n + x + h] = o[u][1];
    buf[(y + h) * n + x] = o[u][2];
    buf[(y + h) * n + x + h] = o[u][3];
  }
  __syncthreads();
}

// Inverse of haar_level_analysis (the 4 x 4 map is its own inverse).
template <int kMaxPer>
__device__ void haar_level_synthesis(float2 *buf, int n, int m) {
  const int h = m >> 1;
  const int nblk = h * h;
  float2 o[kMaxPer][4];
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q >= nblk) break;
    const int y = q / h, x = q % h;
    const float2 ll = buf[y * n + x];
    const float2 tr = buf[y * n + x + h];
    const float2 bl = buf[(y + h) * n + x];
    const float2 hh = buf[(y + h) * n + x + h];
    o[u][0] = make_float2(0.5f * ((ll.x + tr.x) + (bl.x + hh.x)), 0.5f * ((ll.y + tr.y) + (bl.y + hh.y)));
    o[u][1] = make_float2(0.5f * ((ll.x - tr.x) + (bl.x - hh.x)), 0.5f * ((ll.y - tr.y) + (bl.y - hh.y)));
    o[u][2] = make_float2(0.5f * ((ll.x + tr.x) - (bl.x + hh.x)), 0.5f * ((ll.y + tr.y) - (bl.y + hh.y)));
    o[u][3] = make_float2(0.5f * ((ll.x - tr.x) - (bl.x - hh.x)), 0.5f * ((ll.y - tr.y) - (bl.y - hh.y)));
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q >= nblk) break;
    const int y = q / h, x = q % h;
    buf[(2 * y) * n + 2 * x] = o[u][0];
    buf[(2 * y) * n + 2 * x + 1] = o[u][1];
    buf[(2 * y + 1) * n + 2 * x] = o[u][2];
    buf[(2 * y + 1) * n + 2 * x + 1] = o[u][3];
  }
  __syncthreads();
}

constexpr int kHaarThreads = 1024;
constexpr int kHaarMaxN = 8192;  // 64 KB of LDS per row image
constexpr int kHaarMaxPer = kHaarMaxN / 4 / kHaarThreads;  // 2x2 blocks per thread

// A_s = F_s W for the Haar dictionary: one workgroup per frequency row; the
// row, viewed as an n x n image, is formed in LDS and analysed level by level
// (W^T applied to each row, since W is the orthonormal synthesis matrix).
__global__ __launch_bounds__(kHaarThreads) void k_rows_haar(Geom g,
                                                            const double *__restrict__ pos,
                                                            int s, int levels,
                                                            float2 *__restrict__ A) {
  extern __shared__ float2 buf[];
  const int k = blockIdx.x;
  const double c4f = (4.0 * kPi / kC0) * (g.f0 + k * g.df);
  const double *p = pos + 3 * s;
  for (int i = threadIdx.x; i < g.N; i += kHaarThreads) {
    buf[i] = phasor_neg(c4f * pixel_range(g, p, i));
  }
  __syncthreads();
  for (int lev = 0; lev < levels; ++lev) haar_level_analysis<kHaarMaxPer>(buf, g.nx, g.nx >> lev);
  float2 *out = A + static_cast<size_t>(k) * g.Npad;
  for (int i = threadIdx.x; i < g.Npad; i += kHaarThreads)
    out[i] = i < g.N ? buf[i] : make_float2(0.f, 0.f);
}

// x = W c for the Haar dictionary (single workgroup).
__global__ __launch_bounds__(kHaarThreads) void k_image_haar(Geom g, int levels,
                                                             const float2 *__restrict__ c,
                                                             float2 *__restrict__ x) {
  extern __shared__ float2 buf[];
  for (int i = threadIdx.x; i < g.N; i += kHaarThreads) buf[i] = c[i];
  __syncthreads();
  for (int lev = levels - 1; lev >= 0; --lev) haar_level_synthesis<kHaarMaxPer>(buf, g.nx, g.nx >> lev);
  for (int i = threadIdx.x; i < g.N; i += kHaarThreads) x[i] = buf[i];
}

// c = W^T x for the Haar dictionary (analysis of one image; single workgroup).
__global__ __launch_bounds__(kHaarThreads) void k_analysis_haar(Geom g, int levels,
                                                                const float2 *__restrict__ x,
                                                                float2 *__restrict__ c) {
  extern __shared__ float2 buf[];
  for (int i = threadIdx.x; i < g.N; i += kHaarThreads) buf[i] = x[i];
  __syncthreads();
  for (int lev = 0; lev < levels; ++lev) haar_level_analysis<kHaarMaxPer>(buf, g.nx, g.nx >> lev);
  for (int i = threadIdx.x; i < g.Npad; i += kHaarThreads) c[i] = i < g.N ? buf[i] : make_float2(0.f, 0.f);
}

__global__ void k_copy_pad_c64(const float2 *__restrict__ src, float2 *__restrict__ dst, int n, int npad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npad) dst[i] = i < n ? src[i] : make_float2(0.f, 0.f);
}

__global__ void k_copy_c64(const float2 *__restrict__ src, float2 *__restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Fixed-order tree sum over a 256-thread block of double2 values.
__device__ double2 block_sum_d2(double2 v, double2 *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[threadIdx.x].x += red[threadIdx.x + off].x;
      red[threadIdx.x].y += red[threadIdx.x + off].y;
    }
    __syncthreads();
  }
  const double2 r = red[0];
  __syncthreads();
  return r;
}

// Clean echo sum_i F_s[k, i] rho_i, one workgroup per frequency (FP64 sums).
__global__ __launch_bounds__(256) void k_echo_clean(Geom g, const double *__restrict__ pos,
                                                    int s, const float2 *__restrict__ rho,
                                                    double2 *__restrict__ tmp) {
  __shared__ double2 red[256];
  const int k = blockIdx.x;
  const double c4f = (4.0 * kPi / kC0) * (g.f0 + k * g.df);
  const double *p = pos + 3 * s;
  double2 acc = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < g.npix; i += 256) {
    const float2 r = rho[i];
    if (r.x == 0.f && r.y == 0.f) continue;
    const float2 e = phasor_neg(c4f * pixel_range(g, p, i));
    acc.x += static_cast<double>(e.x) * r.x - static_cast<double>(e.y) * r.y;
    acc.y += static_cast<double>(e.x) * r.y + static_cast<double>(e.y) * r.x;
  }
  const double2 t = block_sum_d2(acc, red);
  if (threadIdx.x == 0) tmp[k] = t;
}

// d = exp(i phase_err) clean + sigma noise, sigma^2 = |clean|^2 / K 10^(-snr/10).
__global__ __launch_bounds__(256) void k_echo_finish(int K, const double2 *__restrict__ tmp,
                                                     const float2 *__restrict__ noise,
                                                     double snr_db, double cph, double sph,
                                                     float2 *__restrict__ out) {
  __shared__ double2 red[256];
  double2 e = make_double2(0.0, 0.0);
  for (int k = threadIdx.x; k < K; k += 256) e.x += tmp[k].x * tmp[k].x + tmp[k].y * tmp[k].y;
  const double energy = block_sum_d2(e, red).x;
  const double sigma = noise ? sqrt(energy / K * pow(10.0, -snr_db / 10.0)) : 0.0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const double2 c = tmp[k];
    double re = cph * c.x - sph * c.y;
    double im = cph * c.y + sph * c.x;
    if (noise) {
      re += sigma * noise[k].x;
      im += sigma * noise[k].y;
    }
    out[k] = make_float2(static_cast<float>(re), static_cast<float>(im));
  }
}

constexpr int kToepDCh = 8;  // lags per workgroup

// Toeplitz generator of A_s A_s^H for a uniform frequency grid:
// (A_s A_s^H)[k, l] = g(k - l), g(d) = sum_i exp(-i 4 pi d df R_i / c0), g(-d) = conj(g(d)).
// W W^T = I for both dictionaries, so the pixel-domain kernel suffices.  The
// phasors are FP64: the first lag of a thread's chunk from an FP64 sincos of
// its whole phase (at most ~2e5 rad, so ~2e-11 rad of rounding), the next ones
// by multiplying with the one-lag phasor (one rounding each).
__global__ __launch_bounds__(256) void k_toeplitz(Geom g, const double *__restrict__ pos,
                                                  double2 *__restrict__ gtoep) {
  __shared__ double2 red[256];
  const int s = blockIdx.x;
  const int d0 = blockIdx.y * kToepDCh;
  const double *p = pos + 3 * s;
  const double c4d = 4.0 * kPi / kC0 * g.df;
  double2 acc[kToepDCh];
#pragma unroll
  for (int j = 0; j < kToepDCh; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < g.npix; i += 256) {
    const double th = c4d * pixel_range(g, p, i);
    double s1, c1, s0, c0;
    sincos(th, &s1, &c1);
    sincos(th * d0, &s0, &c0);
    double er = c0, ei = -s0;  // exp(-i d0 th)
#pragma unroll
    for (int j = 0; j < kToepDCh; ++j) {
      acc[j].x += er;
      acc[j].y += ei;
      const double nr = er * c1 + ei * s1;  // times exp(-i th)
      const double ni = ei * c1 - er * s1;
      er = nr;
      ei = ni;
    }
  }
  for (int j = 0; j < kToepDCh; ++j) {
    const double2 t = block_sum_d2(acc[j], red);
    if (threadIdx.x == 0 && d0 + j < g.K) gtoep[static_cast<size_t>(s) * g.K + d0 + j] = t;
  }
}

// ---------------------------------------------------------------------------
// sigma^2 = ||A_s||_2^2 = lambda_max(T) exactly (to FP64 rounding), by
// bisection on mu with the test "mu I - T is positive definite".  The top of
// this spectrum is tightly clustered (lambda_2 / lambda_1 ~ 1 - 1e-7 on the
// workload geometries), which rules out power iteration.  The bracket's upper
// end is returned, so the result is an upper bound up to the rounding of the
// test.

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// mu I - T positive definite?  T Hermitian Toeplitz with first column r
// (T[k, 0] = r[k]).  Levinson-Durbin on S = mu I - T: the prediction-error
// powers E_k are the pivots of S = L D L^H, so S is positive definite exactly
// when every E_k > 0; the recursion stops at the first E_k <= 0 (only the
// leading minors up to that order were needed, and they were definite, so the
// recursion was stable up to there).  One wavefront; a (the predictor,
// a[1..K-1]) lives in LDS and is updated in pairs (j, k - j), one lane per
// pair.
__device__ bool levinson_definite(int K, const double2 *__restrict__ r, double mu,
                                  double2 *__restrict__ a, int lane) {
  double E = mu - r[0].x;
  if (!(E > 0.0)) return false;
  for (int k = 1; k < K; ++k) {
    // acc = s(k) + sum_{j=1}^{k-1} a_j s(k - j),  s(d) = -r(d) for d >= 1
    double pr = 0.0, pi = 0.0;
    for (int j = 1 + lane; j < k; j += 64) {
      const double2 x = a[j], y = r[k - j];
      pr -= x.x * y.x - x.y * y.y;
      pi -= x.x * y.y + x.y * y.x;
    }
    pr = wave_sum_f64(pr) - r[k].x;
    pi = wave_sum_f64(pi) - r[k].y;
    const double kr = -pr / E, ki = -pi / E;  // kappa = -acc / E
    const double m2 = kr * kr + ki * ki;
    const double En = E * (1.0 - m2);
    // a_j <- a_j + kappa conj(a_{k-j}), j = 1..k-1, then a_k = kappa
    for (int j = 1 + lane; 2 * j <= k; j += 64) {
      const int jj = k - j;
      const double2 x = a[j];
      if (jj == j) {
        a[j] = make_double2(x.x + kr * x.x + ki * x.y, x.y + ki * x.x - kr * x.y);
      } else {
        const double2 y = a[jj];
        a[j] = make_double2(x.x + kr * y.x + ki * y.y, x.y + ki * y.x - kr * y.y);
        a[jj] = make_double2(y.x + kr * x.x + ki * x.y, y.y + ki * x.x - kr * x.y);
      }
    }
    if (lane == 0) a[k] = make_double2(kr, ki);
    wave_sync_lds();
    E = En;
    if (!(E > 0.0)) return false;
  }
  return true;
}

constexpr int kSectWaves = 4;     // trial points per bisection round at most (one per wave)
constexpr int kSectRounds = 96;   // rounds at most (a 3-section gains 1.58 bits per round)
constexpr size_t kSectLds = 60 * 1024;  // dynamic LDS budget (generator + predictors)

// Trial waves that fit the LDS budget next to the K-entry generator.
inline int sect_waves(int K) {
  const size_t per = static_cast<size_t>(K) * sizeof(double2);
  const int fit = static_cast<int>(kSectLds / per) - 1;
  return fit < 1 ? 1 : (fit > kSectWaves ? kSectWaves : fit);
}

// One workgroup per position.  Bracket: lambda_max >= T[0, 0]; every row sum
// of |T| is at most |g(0)| + 2 sum_{d >= 1} |g(d)|.  Each round the first nw
// waves test the nw interior points of an (nw + 1)-section and the bracket
// shrinks to the first definite one.
__global__ __launch_bounds__(256) void k_sigma2_toeplitz(int K, int nw,
                                                         const double2 *__restrict__ gtoep,
                                                         double *__restrict__ sig2) {
  extern __shared__ double2 sh[];
  double2 *r = sh;                                      // K
  double2 *apred = sh + K + (threadIdx.x >> 6) * K;     // K per trial wave
  __shared__ double red[256];
  __shared__ int pd[kSectWaves];
  const int s = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double gs = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const double2 v = gtoep[static_cast<size_t>(s) * K + k];
    r[k] = v;
    gs += (k == 0 ? 1.0 : 2.0) * sqrt(v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = gs;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  double lo = r[0].x;
  double hi = red[0] * (1.0 + 1e-14);
  __syncthreads();
  for (int round = 0; round < kSectRounds && hi - lo > 1e-15 * hi; ++round) {
    if (wave < nw) {
      const double mu = lo + (hi - lo) * (wave + 1) / (nw + 1);
      const bool ok = mu > lo && mu < hi ? levinson_definite(K, r, mu, apred, lane) : mu >= hi;
      if (lane == 0) pd[wave] = ok ? 1 : 0;
    }
    __syncthreads();
    int w = 0;
    while (w < nw && !pd[w]) ++w;
    const double nlo = w == 0 ? lo : lo + (hi - lo) * w / (nw + 1);
    const double nhi = w == nw ? hi : lo + (hi - lo) * (w + 1) / (nw + 1);
    __syncthreads();
    if (!(nlo > lo || nhi < hi)) break;  // no representable progress left
    lo = nlo;
    hi = nhi;
  }
  if (threadIdx.x == 0) sig2[s] = hi;
}

// ---------------------------------------------------------------------------
// Edgelet dictionary (Section III-A): binary atoms, so A_s = F_s W is a
// gather-sum of phasors and x = W c, c = W^T x are gather-sums too.

// A_s[k, m] = sum over the pixels p of atom m of exp(-i 4 pi f_k R_p / c0):
// thread per atom, kRowsKCh frequencies per thread; the FP64 range of each
// pixel is formed once per thread and the phasors are added in pixel order.
__global__ __launch_bounds__(256) void k_rows_edgelet(Geom g, const double *__restrict__ pos,
                                                      int s, const int *__restrict__ atom_ptr,
                                                      const int *__restrict__ atom_pix,
                                                      float2 *__restrict__ A) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  const int k0 = blockIdx.y * kRowsKCh;
  if (m >= g.Npad) return;
  const int kn = min(kRowsKCh, g.K - k0);
  float2 *out = A + static_cast<size_t>(k0) * g.Npad + m;
  float2 acc[kRowsKCh];
#pragma unroll
  for (int kk = 0; kk < kRowsKCh; ++kk) acc[kk] = make_float2(0.f, 0.f);
  if (m < g.N) {
    const double c4 = 4.0 * kPi / kC0;
    for (int q = atom_ptr[m]; q < atom_ptr[m + 1]; ++q) {
      const double R = pixel_range(g, pos + 3 * s, atom_pix[q]);
#pragma unroll
      for (int kk = 0; kk < kRowsKCh; ++kk) {
        if (kk < kn) {
          const float2 e = phasor_neg((c4 * (g.f0 + (k0 + kk) * g.df)) * R);
          acc[kk].x += e.x;
          acc[kk].y += e.y;
        }
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < kRowsKCh; ++kk)
    if (kk < kn) out[static_cast<size_t>(kk) * g.Npad] = acc[kk];
}

// x_p = sum of c_m over the atoms m containing pixel p (increasing m).
__global__ __launch_bounds__(256) void k_image_edgelet(int npix, const int *__restrict__ pix_ptr,
                                                       const int *__restrict__ pix_atom,
                                                       const float2 *__restrict__ c,
                                                       float2 *__restrict__ x) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int q = pix_ptr[p]; q < pix_ptr[p + 1]; ++q) {
    const float2 v = c[pix_atom[q]];
    acc.x += v.x;
    acc.y += v.y;
  }
  x[p] = acc;
}

// c_m = sum of x_p over the pixels p of atom m (increasing p); 0 past M.
__global__ __launch_bounds__(256) void k_image_adjoint_edgelet(int M, int Npad,
                                                               const int *__restrict__ atom_ptr,
                                                               const int *__restrict__ atom_pix,
                                                               const float2 *__restrict__ x,
                                                               float2 *__restrict__ c) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= Npad) return;
  float2 acc = make_float2(0.f, 0.f);
  if (m < M) {
    for (int q = atom_ptr[m]; q < atom_ptr[m + 1]; ++q) {
      const float2 v = x[atom_pix[q]];
      acc.x += v.x;
      acc.y += v.y;
    }
  }
  c[m] = acc;
}

// BP accumulation (Section IV-A baseline): thread per pixel, the rotated
// pulse staged in LDS; conj(F) = exp(+i 4 pi f R / c0) with the FP64 phase.
__global__ __launch_bounds__(256) void k_backproject(Geom g, const double *__restrict__ pos, int s,
                                                     const float2 *__restrict__ d, float cphi,
                                                     float sphi, float2 *__restrict__ bp) {
  extern __shared__ float2 dr[];  // K rotated samples
  for (int k = threadIdx.x; k < g.K; k += 256) {
    const float2 v = d[k];
    // d e^{-i phi}
    dr[k] = make_float2(v.x * cphi + v.y * sphi, v.y * cphi - v.x * sphi);
  }
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= g.npix) return;
  const double R = pixel_range(g, pos + 3 * s, p);
  const double c4 = 4.0 * kPi / kC0;
  float re = 0.f, im = 0.f;
  for (int k = 0; k < g.K; ++k) {
    const float2 f = phasor_neg((c4 * (g.f0 + k * g.df)) * R);  // F[k, p]
    const float2 x = dr[k];
    // conj(f) * x
    re += f.x * x.x + f.y * x.y;
    im += f.x * x.y - f.y * x.x;
  }
  float2 acc = bp[p];
  acc.x += re;
  acc.y += im;
  bp[p] = acc;
}

constexpr int kKKB = 16;   // G block edge
constexpr int kKKM = 64;   // coefficients staged per step

// G = A A^H (K x K) with FP64 sums over the M coefficients in increasing
// order: G[k, l] = sum_m A[k, m] conj(A[l, m]).  Workgroup = 16 x 16 block.
__global__ __launch_bounds__(256) void k_gram_kk(int K, int Npad, int M,
                                                 const float2 *__restrict__ A,
                                                 double2 *__restrict__ G) {
  __shared__ float2 ak[kKKB][kKKM + 1];
  __shared__ float2 al[kKKB][kKKM + 1];
  const int tx = threadIdx.x % kKKB, ty = threadIdx.x / kKKB;
  const int k = blockIdx.x * kKKB + ty, l = blockIdx.y * kKKB + tx;
  double re = 0.0, im = 0.0;
  for (int m0 = 0; m0 < M; m0 += kKKM) {
    for (int e = threadIdx.x; e < kKKB * kKKM; e += 256) {
      const int r = e / kKKM, q = e % kKKM;
      const int kr = blockIdx.x * kKKB + r, lr = blockIdx.y * kKKB + r, m = m0 + q;
      ak[r][q] = (kr < K && m < M) ? A[static_cast<size_t>(kr) * Npad + m] : make_float2(0.f, 0.f);
      al[r][q] = (lr < K && m < M) ? A[static_cast<size_t>(lr) * Npad + m] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 8
    for (int q = 0; q < kKKM; ++q) {
      const float2 a = ak[ty][q], b = al[tx][q];
      // a * conj(b)
      re += static_cast<double>(a.x) * b.x + static_cast<double>(a.y) * b.y;
      im += static_cast<double>(a.y) * b.x - static_cast<double>(a.x) * b.y;
    }
    __syncthreads();
  }
  if (k < K && l < K) G[static_cast<size_t>(k) * K + l] = make_double2(re, im);
}

// sigma^2 = lambda_max(G) for a dense Hermitian K x K matrix (the edgelet
// dictionary, where A_s A_s^H is not Toeplitz): Householder reduction to a
// Hermitian tridiagonal matrix in FP64, in place, then bisection on the
// Sturm count of the equivalent real tridiagonal (off-diagonals |e_k|).  One
// workgroup per matrix.  Step k reflects the column below the diagonal,
// x = G[k+1:, k], onto alpha e_1 with alpha = -e^{i arg x_0} |x|:
// v = x - alpha e_1, beta = 2 / |v|^2, p = beta G22 v, w = p - (beta/2)(v^H p) v,
// G22 <- G22 - v w^H - w v^H.  Only the trailing block is kept up to date.
__global__ __launch_bounds__(256) void k_sigma2_dense(int K, double2 *__restrict__ Gall,
                                                      double *__restrict__ sig2) {
  extern __shared__ double2 sh[];
  double2 *v = sh;                                       // K
  double2 *w = sh + K;                                   // K
  double *dg = reinterpret_cast<double *>(sh + 2 * K);   // K diagonal
  double *e2 = dg + K;                                   // K squared off-diagonals
  __shared__ double2 red[256];
  __shared__ double bounds[2];
  double2 *G = Gall + static_cast<size_t>(blockIdx.x) * K * K;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k + 2 < K; ++k) {
    const int m0 = k + 1;
    // x_i = G[i, k] = conj(G[k, i]) (row k is contiguous)
    double2 part = make_double2(0.0, 0.0);
    for (int i = m0 + threadIdx.x; i < K; i += 256) {
      const double2 g = G[static_cast<size_t>(k) * K + i];
      v[i] = make_double2(g.x, -g.y);
      part.x += g.x * g.x + g.y * g.y;
    }
    const double xn2 = block_sum_d2(part, red).x;  // also orders the v stores
    const double2 x0 = v[m0];
    const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    if (threadIdx.x == 0) {
      dg[k] = G[static_cast<size_t>(k) * K + k].x;
      e2[k] = xn2;
    }
    if (!(xn2 - a0 * a0 > 0.0)) {  // already tridiagonal in this column
      __syncthreads();
      continue;
    }
    const double xn = sqrt(xn2);
    const double ur = a0 > 0.0 ? x0.x / a0 : 1.0, ui = a0 > 0.0 ? x0.y / a0 : 0.0;
    const double beta = 1.0 / (xn2 + xn * a0);  // 2 / |v|^2
    __syncthreads();
    if (threadIdx.x == 0) v[m0] = make_double2(x0.x + ur * xn, x0.y + ui * xn);
    __syncthreads();
    // p = beta G22 v: wave per row, lanes along the row
    for (int i = m0 + wave; i < K; i += 4) {
      double re = 0.0, im = 0.0;
      for (int j = m0 + lane; j < K; j += 64) {
        const double2 g = G[static_cast<size_t>(i) * K + j], y = v[j];
        re += g.x * y.x - g.y * y.y;
        im += g.x * y.y + g.y * y.x;
      }
      re = wave_sum_f64(re);
      im = wave_sum_f64(im);
      if (lane == 0) w[i] = make_double2(beta * re, beta * im);
    }
    __syncthreads();
    part = make_double2(0.0, 0.0);
    for (int i = m0 + threadIdx.x; i < K; i += 256)  // Re(v^H p)
      part.x += v[i].x * w[i].x + v[i].y * w[i].y;
    const double kc = 0.5 * beta * block_sum_d2(part, red).x;
    for (int i = m0 + threadIdx.x; i < K; i += 256)
      w[i] = make_double2(w[i].x - kc * v[i].x, w[i].y - kc * v[i].y);
    __syncthreads();
    // G22 -= v w^H + w v^H
    const int m = K - m0;
    for (int e = threadIdx.x; e < m * m; e += 256) {
      const int i = m0 + e / m, j = m0 + e % m;
      const double2 vi = v[i], wi = w[i], vj = v[j], wj = w[j];
      double2 &g = G[static_cast<size_t>(i) * K + j];
      g.x -= (vi.x * wj.x + vi.y * wj.y) + (wi.x * vj.x + wi.y * vj.y);
      g.y -= (vi.y * wj.x - vi.x * wj.y) + (wi.y * vj.x - wi.x * vj.y);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (K >= 2) {
      const double2 g = G[static_cast<size_t>(K - 1) * K + (K - 2)];
      dg[K - 2] = G[static_cast<size_t>(K - 2) * K + (K - 2)].x;
      e2[K - 2] = g.x * g.x + g.y * g.y;
    }
    dg[K - 1] = G[static_cast<size_t>(K - 1) * K + (K - 1)].x;
    // bracket: lambda_max >= max diagonal; Gershgorin for the upper end
    double lo = dg[0], hi = -1e300;
    for (int i = 0; i < K; ++i) {
      const double el = i > 0 ? sqrt(e2[i - 1]) : 0.0, er = i + 1 < K ? sqrt(e2[i]) : 0.0;
      lo = fmax(lo, dg[i]);
      hi = fmax(hi, dg[i] + el + er);
    }
    bounds[0] = lo;
    bounds[1] = hi * (1.0 + 1e-14) + 1e-300;
  }
  __syncthreads();
  // 256-section rounds: thread t tests lo + (hi - lo)(t + 1)/257 with the
  // Sturm count (number of eigenvalues below mu = number of negative pivots
  // of T - mu I); "all K below" means mu is above lambda_max.
  __shared__ int below[256];
  double lo = bounds[0], hi = bounds[1];
  for (int round = 0; round < 12 && hi - lo > 1e-15 * fabs(hi); ++round) {
    const double mu = lo + (hi - lo) * (threadIdx.x + 1) / 257.0;
    int cnt = 0;
    double q = dg[0] - mu;
    const double tiny = 1e-300;
    if (q == 0.0) q = -tiny;
    cnt += q < 0.0;
    for (int i = 1; i < K; ++i) {
      q = dg[i] - mu - e2[i - 1] / q;
      if (q == 0.0) q = -tiny;
      cnt += q < 0.0;
    }
    below[threadIdx.x] = (mu > lo && mu < hi) ? (cnt == K) : (mu >= hi);
    __syncthreads();
    int t = 0;
    while (t < 256 && !below[t]) ++t;
    const double nlo = t == 0 ? lo : lo + (hi - lo) * t / 257.0;
    const double nhi = t == 256 ? hi : lo + (hi - lo) * (t + 1) / 257.0;
    __syncthreads();
    if (!(nlo > lo || nhi < hi)) break;
    lo = nlo;
    hi = nhi;
  }
  if (threadIdx.x == 0) sig2[blockIdx.x] = hi;
}

}  // namespace

hipError_t launch_rows(const Geom &g, const double *pos, int s, float2 *A,
                       const DictTabs &dt, hipStream_t st) {
  if (dt.kind == 1) {
    const size_t lds = static_cast<size_t>(g.N) * sizeof(float2);
    hipLaunchKernelGGL(k_rows_haar, dim3(g.K), dim3(kHaarThreads), lds, st, g, pos, s, dt.levels, A);
  } else if (dt.kind == 2) {
    dim3 grid((g.Npad + 255) / 256, (g.K + kRowsKCh - 1) / kRowsKCh);
    hipLaunchKernelGGL(k_rows_edgelet, grid, dim3(256), 0, st, g, pos, s, dt.atom_ptr, dt.atom_pix, A);
  } else {
    dim3 grid((g.Npad + 255) / 256, (g.K + kRowsKCh - 1) / kRowsKCh);
    hipLaunchKernelGGL(k_rows_identity, grid, dim3(256), 0, st, g, pos, s, A);
  }
  return hipGetLastError();
}

hipError_t launch_image(const Geom &g, const float2 *c, float2 *x, const DictTabs &dt,
                        hipStream_t st) {
  if (dt.kind == 1) {
    const size_t lds = static_cast<size_t>(g.N) * sizeof(float2);
    hipLaunchKernelGGL(k_image_haar, dim3(1), dim3(kHaarThreads), lds, st, g, dt.levels, c, x);
  } else if (dt.kind == 2) {
    hipLaunchKernelGGL(k_image_edgelet, dim3((g.npix + 255) / 256), dim3(256), 0, st, g.npix,
                       dt.pix_ptr, dt.pix_atom, c, x);
  } else {
    hipLaunchKernelGGL(k_copy_c64, dim3((g.N + 255) / 256), dim3(256), 0, st, c, x, g.N);
  }
  return hipGetLastError();
}

hipError_t launch_image_adjoint(const Geom &g, const float2 *x, float2 *c, const DictTabs &dt,
                                hipStream_t st) {
  if (dt.kind == 1) {
    const size_t lds = static_cast<size_t>(g.N) * sizeof(float2);
    hipLaunchKernelGGL(k_analysis_haar, dim3(1), dim3(kHaarThreads), lds, st, g, dt.levels, x, c);
  } else if (dt.kind == 2) {
    hipLaunchKernelGGL(k_image_adjoint_edgelet, dim3((g.Npad + 255) / 256), dim3(256), 0, st, g.N,
                       g.Npad, dt.atom_ptr, dt.atom_pix, x, c);
  } else {
    hipLaunchKernelGGL(k_copy_pad_c64, dim3((g.Npad + 255) / 256), dim3(256), 0, st, x, c, g.N, g.Npad);
  }
  return hipGetLastError();
}

hipError_t launch_backproject(const Geom &g, const double *pos, int s, const float2 *d,
                              double cos_c, double sin_c, float2 *bp, hipStream_t st) {
  const size_t lds = static_cast<size_t>(g.K) * sizeof(float2);
  hipLaunchKernelGGL(k_backproject, dim3((g.npix + 255) / 256), dim3(256), lds, st, g, pos, s, d,
                     static_cast<float>(cos_c), static_cast<float>(sin_c), bp);
  return hipGetLastError();
}

hipError_t launch_echo(const Geom &g, const double *pos, int s,
                       const float2 *rho, const float2 *noise, double snr_db,
                       double phase_err, double2 *tmp, float2 *out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_echo_clean, dim3(g.K), dim3(256), 0, st, g, pos, s, rho, tmp);
  hipLaunchKernelGGL(k_echo_finish, dim3(1), dim3(256), 0, st, g.K, tmp, noise, snr_db,
                     cos(phase_err), sin(phase_err), out);
  return hipGetLastError();
}

hipError_t launch_sigma2(const Geom &g, const double *pos, double2 *gtoep,
                         double *sig2, hipStream_t st) {
  dim3 grid(g.npos, (g.K + kToepDCh - 1) / kToepDCh);
  hipLaunchKernelGGL(k_toeplitz, grid, dim3(256), 0, st, g, pos, gtoep);
  const int nw = sect_waves(g.K);
  const size_t lds = (1 + nw) * static_cast<size_t>(g.K) * sizeof(double2);
  hipLaunchKernelGGL(k_sigma2_toeplitz, dim3(g.npos), dim3(256), lds, st, g.K, nw, gtoep, sig2);
  return hipGetLastError();
}

hipError_t launch_gram_kk(const Geom &g, const float2 *A, double2 *G, hipStream_t st) {
  const int nbk = (g.K + kKKB - 1) / kKKB;
  hipLaunchKernelGGL(k_gram_kk, dim3(nbk, nbk), dim3(256), 0, st, g.K, g.Npad, g.N, A, G);
  return hipGetLastError();
}

hipError_t launch_sigma2_dense(int K, double2 *G, int nmat, double *sig2, hipStream_t st) {
  if (nmat <= 0) return hipSuccess;
  const size_t lds = 2 * static_cast<size_t>(K) * (sizeof(double2) + sizeof(double));
  hipLaunchKernelGGL(k_sigma2_dense, dim3(nmat), dim3(256), lds, st, K, G, sig2);
  return hipGetLastError();
}

}  // namespace ofista
