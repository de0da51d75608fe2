// Sufficient-statistic updates of one pulse (Section III-C):
//   H += A_s^H A_s         (rank-K Hermitian Gram update on the matrix cores)
//   b += A_s^H d~          (correlation, formed by the diagonal-tile workgroups
//                           from the A blocks they already stage; at the first
//                           pulse also max_i |Delta b_i|)
//
// The Gram update is the one dense contraction on the path.  For a tile
// (I, J) of H, with a = A_s[k, I-block] and a' = A_s[k, J-block] complex,
//   Re H_ij += sum_k ar_i ar'_j + ai_i ai'_j,   Im H_ij += sum_k ar_i ai'_j - ai_i ar'_j.
// The FP32 kernel forms these from three real products (Gauss's method for a
// complex product): G1 = (ar - ai) ar', G2 = ar (ai' - ar'), G3 = ai (ar' + ai'),
// Re = G1 + G3, Im = G1 + G2.  v_mfma_f32_32x32x2f32 contracts two terms per
// instruction, here two frequencies, so two frequencies cost three
// instructions instead of the four of the direct form (kept as THREE = false:
// one frequency per instruction with A = (ar, ai)[l/32] and B = (ar', ai') for
// Re, (ai', -ar') for Im).  Only tiles with I <= J exist (packed upper
// storage); the diagonal of each diagonal tile gets Im = 0 exactly.
#include "ofista_internal.h"

namespace ofista {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// H(I, J) += A_I^H A_J for one 64 x 64 tile per workgroup, 4 waves each
// owning a 32 x 32 quadrant; KB frequencies are staged through LDS per step,
// the next step's operands are loaded into registers while the matrix cores
// work on the current one.  Workgroup b runs on XCD b % 8; logical tile
// (b % 8) * per + b / 8 gives each XCD a contiguous run of the tile table,
// whose order (8 x 8 super-tiles) keeps the A blocks of concurrently running
// tiles inside one XCD's L2.
//
// A table entry with a nonzero piece number p is part p of a split tile: it
// contracts only frequency stages [(p-1) nst / parts, p nst / parts) of the
// nst stages and stores its partial to P instead of updating H.
//
// THREE = true: the three-real-product form of the complex product (Gauss).
// With two frequencies per instruction (lane half h takes frequency 2u + h),
//   G1 += (ar_i - ai_i) ar'_j,  G2 += ar_i (ai'_j - ar'_j),  G3 += ai_i (ar'_j + ai'_j),
// and Re = G1 + G3, Im = G1 + G2: three instructions per two frequencies
// instead of four, and one LDS read per operand per two frequencies.
template <int KB, bool THREE>
__global__ __launch_bounds__(256) void k_gram_fp32(int K, int Npad, int ntiles_grid,
                                                   const float2 *__restrict__ A,
                                                   const int2 *__restrict__ tile_ij,
                                                   float2 *__restrict__ H, CorrArgs corr,
                                                   float2 *__restrict__ P, int parts) {
  static_assert(KB % 8 == 0, "two float4 loads per thread per 8 frequencies");
  constexpr int kLoads = KB / 8;  // float4 per thread per operand and step
  __shared__ float2 sa[KB][kTile];
  __shared__ float2 sb[KB][kTile];
  __shared__ float2 sd[kMaxFreq];  // rotated pulse, diagonal tiles only
  const int per = ntiles_grid >> 3;
  const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int2 ij = tile_ij[logical];
  if (ij.x < 0) return;  // padding of the grid to a multiple of 8
  const int I = ij.x & 0xFFFF, J = ij.y & 0xFFFFF;
  const int piece = ij.y >> 20, sidx = ij.x >> 16;
  int kbeg = 0, kend = K;
  if (piece > 0) {
    const int nst = (K + KB - 1) / KB;
    kbeg = (piece - 1) * nst / parts * KB;
    kend = min(K, piece * nst / parts * KB);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const bool hi = lane >= 32;
  const int li = lane & 31;
  // Correlation on the diagonal tiles: b_I += A_I^H d~ from the staged A_I.
  // Thread t sums column t % 64 over frequencies kk in [g KB/4, (g+1) KB/4)
  // of every stage, g = t / 64; the four groups are added in fixed order.
  const bool diag = I == J;
  float2 bacc = make_float2(0.f, 0.f);
  if (diag) {
    for (int k = threadIdx.x; k < K; k += 256) {
      const float2 v = corr.d[k];
      // d e^{-i phi} = (v.x + i v.y)(cos phi - i sin phi)
      sd[k] = make_float2(v.x * corr.cphi + v.y * corr.sphi, v.y * corr.cphi - v.x * corr.sphi);
    }
  }

  floatx16 accR, accI, acc3;  // THREE: G1, G2, G3
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] = 0.f;
    accI[r] = 0.f;
    acc3[r] = 0.f;
  }

  // staging: KB x 64 complex per operand = KB*32 float4; element r of a
  // thread's prefetch is frequency (threadIdx.x + 256 r) / 32 of the step,
  // float4 column (threadIdx.x + 256 r) % 32
  const float4 *Ag = reinterpret_cast<const float4 *>(A);
  const int rowf4 = Npad >> 1;  // float4 per A row
  const int kk0 = threadIdx.x >> 5, c2 = threadIdx.x & 31;
  const float4 *pI = Ag + I * (kTile / 2) + c2;
  const float4 *pJ = Ag + J * (kTile / 2) + c2;
  float4 pa[kLoads], pb[kLoads];
#pragma unroll
  for (int r = 0; r < kLoads; ++r) {
    const int k = kbeg + kk0 + 8 * r;
    const bool in = k < kend;
    pa[r] = in ? pI[static_cast<size_t>(k) * rowf4] : make_float4(0.f, 0.f, 0.f, 0.f);
    pb[r] = in ? pJ[static_cast<size_t>(k) * rowf4] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int r = 0; r < kLoads; ++r) {
    reinterpret_cast<float4 *>(&sa[kk0 + 8 * r][0])[c2] = pa[r];
    reinterpret_cast<float4 *>(&sb[kk0 + 8 * r][0])[c2] = pb[r];
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
    const bool more = k0 + KB < kend;
    if (more) {
#pragma unroll
      for (int r = 0; r < kLoads; ++r) {
        const int k = k0 + KB + kk0 + 8 * r;
        const bool in = k < kend;
        pa[r] = in ? pI[static_cast<size_t>(k) * rowf4] : make_float4(0.f, 0.f, 0.f, 0.f);
        pb[r] = in ? pJ[static_cast<size_t>(k) * rowf4] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if (THREE) {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 2) {
        const float2 a = sa[kk + (hi ? 1 : 0)][wi * 32 + li];
        const float2 c = sb[kk + (hi ? 1 : 0)][wj * 32 + li];
        accR = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x - a.y, c.x, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, c.y - c.x, accI, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, c.x + c.y, acc3, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const float2 a = sa[kk][wi * 32 + li];
        const float2 c = sb[kk][wj * 32 + li];
        const float av = hi ? a.y : a.x;
        const float br = hi ? c.y : c.x;
        const float bi = hi ? -c.x : c.y;
        accR = __builtin_amdgcn_mfma_f32_32x32x2f32(av, br, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bi, accI, 0, 0, 0);
      }
    }
    if (diag) {
      const int cb = threadIdx.x & 63, g = threadIdx.x >> 6;
#pragma unroll
      for (int u = 0; u < KB / 4; ++u) {
        const int kk = g * (KB / 4) + u;
        if (k0 + kk < K) {
          const float2 x = sa[kk][cb];
          const float2 y = sd[k0 + kk];
          // conj(x) * y
          bacc.x += x.x * y.x + x.y * y.y;
          bacc.y += x.x * y.y - x.y * y.x;
        }
      }
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int r = 0; r < kLoads; ++r) {
        reinterpret_cast<float4 *>(&sa[kk0 + 8 * r][0])[c2] = pa[r];
        reinterpret_cast<float4 *>(&sb[kk0 + 8 * r][0])[c2] = pb[r];
      }
      __syncthreads();
    }
  }

  if (diag) {
    // the staging buffers are free after the last stage's barrier
    float2 *part = &sa[0][0];  // [4][64]
    float *mag = reinterpret_cast<float *>(&sb[0][0]);
    part[threadIdx.x] = bacc;
    __syncthreads();
    if (threadIdx.x < 64) {
      float2 db = part[threadIdx.x];
#pragma unroll
      for (int g = 1; g < 4; ++g) {
        db.x += part[threadIdx.x + 64 * g].x;
        db.y += part[threadIdx.x + 64 * g].y;
      }
      const int i = I * kTile + threadIdx.x;
      float2 bi = corr.b[i];
      bi.x += db.x;
      bi.y += db.y;
      corr.b[i] = bi;
      mag[threadIdx.x] = sqrtf(db.x * db.x + db.y * db.y);
    }
    if (corr.first) {
      __syncthreads();
      if (threadIdx.x == 0) {
        float m = 0.f;
        for (int q = 0; q < 64; ++q) m = fmaxf(m, mag[q]);
        // max of non-negative floats: integer order equals float order
        atomicMax(&corr.scal->dbmax_bits, __float_as_uint(m));
      }
    }
  }

  if (THREE) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float g1 = accR[r];
      accR[r] = g1 + acc3[r];
      accI[r] = g1 + accI[r];
    }
  }
  // epilogue: read-modify-write of the packed tile.  Accumulator register r of
  // lane l holds row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the quadrant.
  if (piece > 0) {
    float2 *Pt = P + (static_cast<size_t>(sidx) * parts + (piece - 1)) * (kTile * kTile);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      Pt[row * kTile + wj * 32 + li] = make_float2(accR[r], accI[r]);
    }
    return;
  }
  const int nb = Npad / kTile;
  const size_t tile_index = static_cast<size_t>(I) * nb - static_cast<size_t>(I) * (I - 1) / 2 + (J - I);
  float2 *Ht = H + tile_index * (kTile * kTile);
  float2 h[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    h[r] = Ht[row * kTile + wj * 32 + li];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int col = wj * 32 + li;
    h[r].x += accR[r];
    h[r].y += accI[r];
    if (I == J && row == col) h[r].y = 0.f;
    Ht[row * kTile + col] = h[r];
  }
}

// H(I, J) += sum over pieces p = 0..parts-1 of P[s][p], in increasing p, for
// split tile s = blockIdx.x; 16 workgroups of 256 elements per tile.  With
// SCAL, workgroup (nsplit, 0) of a grid one column wider runs the pulse
// scalars instead (they read only what earlier launches wrote).
template <bool SCAL>
__global__ __launch_bounds__(256) void k_gram_fixup(int nb, int parts, const int2 *__restrict__ ij,
                                                    const float2 *__restrict__ P,
                                                    float2 *__restrict__ H, ScalarArgs sc) {
  const int s = blockIdx.x;
  if (SCAL && s == static_cast<int>(gridDim.x) - 1) {
    __shared__ double red[256];
    if (blockIdx.y == 0) pulse_scalars(sc, red);
    return;
  }
  const int e = blockIdx.y * 256 + threadIdx.x;
  // all pieces are loaded at once (indices clamped to the last piece), and H
  // as soon as the tile's position is known; summed in increasing p
  const int2 tij = ij[s];
  const float2 *q = P + static_cast<size_t>(s) * parts * (kTile * kTile) + e;
  float2 v[kGramSplitMaxParts];
#pragma unroll
  for (int p = 0; p < kGramSplitMaxParts; ++p)
    v[p] = q[static_cast<size_t>(p < parts ? p : parts - 1) * (kTile * kTile)];
  const int I = tij.x, J = tij.y;
  const size_t tile_index = static_cast<size_t>(I) * nb - static_cast<size_t>(I) * (I - 1) / 2 + (J - I);
  float2 *h = H + tile_index * (kTile * kTile) + e;
  float2 hv = *h;
  float2 acc = v[0];
#pragma unroll
  for (int p = 1; p < kGramSplitMaxParts; ++p) {
    if (p < parts) {
      acc.x += v[p].x;
      acc.y += v[p].y;
    }
  }
  hv.x += acc.x;
  hv.y += acc.y;
  *h = hv;
}

constexpr int kCorrPix = 32;    // pixels per workgroup
constexpr int kCorrGroups = 8;  // frequency groups per workgroup (k = g, g+8, ...)

// b += A^H (d e^{-i phi}); at the first pulse also max_i |Delta b_i| for
// lambda.  Workgroup = 32 pixels x 8 frequency groups; the 8 group sums are
// added in fixed order.
__global__ __launch_bounds__(256) void k_corr(Geom g, const float2 *__restrict__ A,
                                              const float2 *__restrict__ d,
                                              float cphi, float sphi,
                                              float2 *__restrict__ b,
                                              DevScalars *__restrict__ scal, int first,
                                              float2 *__restrict__ delta) {
  extern __shared__ float2 dl[];  // K rotated samples
  __shared__ float2 part[kCorrGroups][kCorrPix];
  __shared__ float red[kCorrPix];
  for (int k = threadIdx.x; k < g.K; k += 256) {
    const float2 v = d[k];
    // d e^{-i phi} = (v.x + i v.y)(cos phi - i sin phi)
    dl[k] = make_float2(v.x * cphi + v.y * sphi, v.y * cphi - v.x * sphi);
  }
  __syncthreads();
  const int px = threadIdx.x & (kCorrPix - 1);
  const int grp = threadIdx.x / kCorrPix;
  const int i = blockIdx.x * kCorrPix + px;  // < Npad (Npad is a multiple of 64)
  float re = 0.f, im = 0.f;
#pragma unroll 8
  for (int k = grp; k < g.K; k += kCorrGroups) {
    const float2 a = A[static_cast<size_t>(k) * g.Npad + i];
    const float2 x = dl[k];
    // conj(a) * x
    re += a.x * x.x + a.y * x.y;
    im += a.x * x.y - a.y * x.x;
  }
  part[grp][px] = make_float2(re, im);
  __syncthreads();
  if (grp == 0) {
    float2 s = part[0][px];
#pragma unroll
    for (int q = 1; q < kCorrGroups; ++q) {
      s.x += part[q][px].x;
      s.y += part[q][px].y;
    }
    if (b) {
      float2 bi = b[i];
      bi.x += s.x;
      bi.y += s.y;
      b[i] = bi;
    }
    if (delta) delta[i] = s;
    red[px] = sqrtf(s.x * s.x + s.y * s.y);
  }
  if (first) {
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = 0.f;
      for (int q = 0; q < kCorrPix; ++q) m = fmaxf(m, red[q]);
      // max of non-negative floats: integer order equals float order
      atomicMax(&scal->dbmax_bits, __float_as_uint(m));
    }
  }
}


// ---------------------------------------------------------------------------
// Precision form: split-BF16 Gram update.  Each FP32 component x of A_s is
// split once per pulse into hi = bf16(x) and lo = bf16(x - hi) (round to
// nearest even).  Per 8 frequencies a wave issues v_mfma_f32_32x32x16_bf16
// three times per plane (hi*hi + hi*lo + lo*hi, the lo*lo term dropped)
// accumulating in FP32: Re uses B = (ar', ai') and Im uses B = (ai', -ar'), as
// in the FP32 kernel.  A and B fragments use the same lane/element-to-k
// assignment, so every (frequency, component) pair is contracted with its own
// partner whatever that assignment is.
//
// Plane layout (hi and lo alike): a word holds one frequency's (re, im) bf16
// pair, re in the low half.  The words are grouped in panel-stage blocks of
// 4 KB, one per 64-pixel panel P and stage s of 16 frequencies, at word
// (P * K/16 + s) * 1024; inside a block, the 16-byte chunk 64 fq + c holds the
// four frequencies 16 s + 4 fq .. +3 of pixel 64 P + c.  A lane's MFMA
// fragment (one pixel, four frequencies) is one chunk, a block is staged into
// LDS as it is, and 16 consecutive lanes read 16 consecutive chunks, so the
// LDS reads are free of bank conflicts.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_to_float(unsigned h) { return __uint_as_float(h << 16); }

constexpr int kSplitTile = 64;
constexpr int kPanelStage = 16;                   // frequencies per panel-stage block
constexpr int kBlockWords = kTile * kPanelStage;  // 1024 words = 4 KB

// A (K x Npad complex64, frequency rows) -> Ahi, Alo in panel-stage blocks.
// One workgroup per 64 pixels x 64 frequencies, transposed through LDS.
__global__ __launch_bounds__(256) void k_split_bf16(int K, int Npad, const float2 *__restrict__ A,
                                                    unsigned *__restrict__ Ahi,
                                                    unsigned *__restrict__ Alo) {
  __shared__ float2 tile[kSplitTile][kSplitTile + 1];
  const int p0 = blockIdx.x * kSplitTile, k0 = blockIdx.y * kSplitTile;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int idx = threadIdx.x + 256 * r;
    const int f = idx >> 6, px = idx & 63;
    tile[f][px] = k0 + f < K ? A[static_cast<size_t>(k0 + f) * Npad + p0 + px] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const size_t nS = static_cast<size_t>(K) / kPanelStage;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int idx = threadIdx.x + 256 * r;
    const int c = idx & 63, quad = idx >> 6;  // quad: 4 frequencies 4 quad .. +3 of the tile
    const int k = k0 + 4 * quad;
    if (k < K) {  // K is a multiple of 16: a chunk is all in or all out
      unsigned hw[4], lw[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const float2 v = tile[4 * quad + w][c];
        const unsigned hr = bf16_rne(v.x), hi = bf16_rne(v.y);
        const unsigned lr = bf16_rne(v.x - bf16_to_float(hr)), li = bf16_rne(v.y - bf16_to_float(hi));
        hw[w] = hr | (hi << 16);
        lw[w] = lr | (li << 16);
      }
      const size_t chunk = ((blockIdx.x * nS + (k >> 4)) * 4 + ((k >> 2) & 3)) * kTile + c;
      typedef unsigned u4 __attribute__((ext_vector_type(4)));
      reinterpret_cast<u4 *>(Ahi)[chunk] = u4{hw[0], hw[1], hw[2], hw[3]};
      reinterpret_cast<u4 *>(Alo)[chunk] = u4{lw[0], lw[1], lw[2], lw[3]};
    }
  }
}

constexpr int kBfKB = 32;  // frequencies per LDS stage of the one-tile kernel (two blocks)

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// (ar, ai) pairs -> (ai, -ar) pairs: the B operand of the imaginary plane.
__device__ __forceinline__ u32x4 im_operand(u32x4 v) {
  return (v >> 16u) | ((v ^ 0x8000u) << 16u);
}

// One 64 x 64 tile per workgroup, 4 waves each owning a 32 x 32 quadrant; a
// stage (two panel-stage blocks per plane and side) is loaded into registers
// while the matrix cores work on the previous one.  Launch order as in the
// FP32 kernel (contiguous runs of the tile table per XCD).
__global__ __launch_bounds__(256) void k_gram_bf16x3(int K, int Npad, int ntiles_grid,
                                                     const unsigned *__restrict__ Ahi,
                                                     const unsigned *__restrict__ Alo,
                                                     const int2 *__restrict__ tile_ij,
                                                     float2 *__restrict__ H) {
  constexpr int kStageChunks = 2 * kBlockWords / 4;  // 512 chunks per plane and side
  __shared__ u32x4 sAh[kStageChunks], sAl[kStageChunks], sBh[kStageChunks], sBl[kStageChunks];
  const int per = ntiles_grid >> 3;
  const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int2 ij = tile_ij[logical];
  if (ij.x < 0) return;
  const int I = ij.x, J = ij.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  floatx16 accR, accI;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] = 0.f;
    accI[r] = 0.f;
  }
  // a stage is 2 consecutive blocks = 512 consecutive chunks per plane and
  // side; thread t moves chunks t and t + 256
  const u32x4 *gAh = reinterpret_cast<const u32x4 *>(Ahi);
  const u32x4 *gAl = reinterpret_cast<const u32x4 *>(Alo);
  const size_t nS = static_cast<size_t>(K) / kPanelStage;
  const size_t baseI = static_cast<size_t>(I) * nS * (kBlockWords / 4) + threadIdx.x;
  const size_t baseJ = static_cast<size_t>(J) * nS * (kBlockWords / 4) + threadIdx.x;
  u32x4 pah[2], pal[2], pbh[2], pbl[2];
  auto fetch = [&](int k0) {
    const size_t o = static_cast<size_t>(k0 >> 4) * (kBlockWords / 4);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      pah[r] = gAh[baseI + o + 256 * r];
      pal[r] = gAl[baseI + o + 256 * r];
      pbh[r] = gAh[baseJ + o + 256 * r];
      pbl[r] = gAl[baseJ + o + 256 * r];
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      sAh[threadIdx.x + 256 * r] = pah[r];
      sAl[threadIdx.x + 256 * r] = pal[r];
      sBh[threadIdx.x + 256 * r] = pbh[r];
      sBl[threadIdx.x + 256 * r] = pbl[r];
    }
  };
  fetch(0);
  stash();
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += kBfKB) {
    const bool more = k0 + kBfKB < K;
    if (more) fetch(k0 + kBfKB);
#pragma unroll
    for (int g = 0; g < kBfKB / 8; ++g) {
      // frequencies 8 g + 4 h .. +3: block g / 2, quad 2 (g % 2) + h
      const int q = (g >> 1) * 256 + (2 * (g & 1) + h) * 64;
      const u32x4 ah = sAh[q + wi * 32 + li];
      const u32x4 al = sAl[q + wi * 32 + li];
      const u32x4 bh = sBh[q + wj * 32 + li];
      const u32x4 bl = sBl[q + wj * 32 + li];
      const bf16x8 Ah = as_bf16x8(ah), Al = as_bf16x8(al);
      const bf16x8 Bh = as_bf16x8(bh), Bl = as_bf16x8(bl);
      const bf16x8 Bhi = as_bf16x8(im_operand(bh)), Bli = as_bf16x8(im_operand(bl));
      accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bhi, accI, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bli, accI, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bhi, accI, 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stash();
      __syncthreads();
    }
  }
  const int nb = Npad / kTile;
  const size_t tile_index = static_cast<size_t>(I) * nb - static_cast<size_t>(I) * (I - 1) / 2 + (J - I);
  float2 *Ht = H + tile_index * (kTile * kTile);
  float2 hv[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    hv[r] = Ht[row * kTile + wj * 32 + li];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int col = wj * 32 + li;
    hv[r].x += accR[r];
    hv[r].y += accI[r];
    if (I == J && row == col) hv[r].y = 0.f;
    Ht[row * kTile + col] = hv[r];
  }
}

// Split-BF16 Gram over 2 x 2 blocks of tiles: wave w owns the whole 64 x 64
// tile (I0 + w/2, J0 + w%2) as 2 x 2 quadrants, so every A fragment read from
// LDS feeds two quadrants and every B fragment two.  A stage is 8 frequencies:
// one half panel-stage block (2 KB) per plane and panel, 8 of them (16 KB),
// moved by direct global-to-LDS loads (global_load_lds_dwordx4: each lane's
// 16 bytes land at the wave's LDS base + 16 lane) into a ring of RING LDS
// buffers, RING - 1 stages ahead of the matrix cores.  No staging registers
// are needed, so two workgroups (two waves per SIMD) fit on a CU.
//
// Per stage: wait until the own loads of this stage have landed (the newer
// stages' loads stay in flight: vmcnt counts the loads in issue order), a
// plain s_barrier (every wave's loads for the stage have landed, and every
// wave has finished reading the buffer the next loads overwrite), read the
// stage's fragments into registers, issue the loads of stage + RING - 1 into
// the buffer read one stage earlier, then run the 24 MFMAs.  __syncthreads()
// is not used: its release fence waits for all loads in flight, which would
// cut the ring to one stage.  The MFMA sequence is the one of the one-tile
// kernel per quadrant, so both layouts give the same H bit for bit.
//
// Block b of the launch takes table entry b; the host orders the table so
// that XCD b % 8 gets a contiguous run of 8 x 8 super-blocks (blocks that
// share panels run on one XCD).
typedef __attribute__((address_space(1))) const void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;

constexpr int kBbRing = 5;         // LDS buffers per workgroup (16 KB each)
constexpr int kBbStageFreq = 8;    // frequencies per stage
constexpr int kBbLoads = 4;        // global_load_lds_dwordx4 per wave per stage

template <int RING>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_gram_bf16_blk(int K, int Npad, const unsigned *__restrict__ Ahi,
                     const unsigned *__restrict__ Alo, const int2 *__restrict__ blocks,
                     float2 *__restrict__ H) {
  constexpr int kSlots = 8;  // [A hi t0, A hi t1, A lo t0, A lo t1, B hi t0, B hi t1, B lo t0, B lo t1]
  constexpr int kSlotChunks = kBlockWords / 8;  // half a block: 128 chunks = 2 KB
  constexpr int kBufChunks = kSlots * kSlotChunks;
  static_assert(RING >= 2 && RING * kBufChunks * 16 <= 80 * 1024, "two workgroups per CU");
  __shared__ u32x4 sbuf[RING * kBufChunks];
  const int2 blk = blocks[blockIdx.x];
  if (blk.x < 0) return;
  const int IB = blk.x, JB = blk.y;
  const int nb = Npad / kTile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = wave >> 1, tj = wave & 1;
  const int I = 2 * IB + ti, J = 2 * JB + tj;
  const bool live = I < nb && J < nb && J >= I;
  const int li = lane & 31, h = lane >> 5;
  floatx16 acc[2][2][2];  // [qi][qj][Re, Im]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[a][b][0][r] = 0.f;
        acc[a][b][1][r] = 0.f;
      }
  // wave w loads slots 2w and 2w + 1: side w / 2, plane w % 2, panels t = 0, 1
  // (the last panel stands in for a missing one of a partial block).  Stage u
  // of panel P is half u % 2 of block (P, u / 2): 512 words at
  // (P K/16 + u/2) 1024 + (u % 2) 512.
  const int nT = K / kBbStageFreq;
  const unsigned *plane = (wave & 1) ? Alo : Ahi;
  const int P0 = 2 * ((wave >> 1) ? JB : IB);
  const unsigned *src[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
    src[t] = plane + static_cast<size_t>(min(P0 + t, nb - 1)) * (K / kPanelStage) * kBlockWords +
             4 * lane;
  auto load_stage = [&](int u, int buf) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        __builtin_amdgcn_global_load_lds(
            (gptr_t)(src[t] + static_cast<size_t>(u) * (kBlockWords / 2) + 256 * j),
            (lptr_t)(&sbuf[buf * kBufChunks + (2 * wave + t) * kSlotChunks + 64 * j]), 16, 0, 0);
  };
  for (int u = 0; u < RING - 1 && u < nT; ++u) load_stage(u, u);
  int rb = 0, wb = RING - 1;  // buffer read at this stage, buffer loaded at this stage
  for (int u = 0; u < nT; ++u) {
    // the loads of stages u + 1 .. u + RING - 2 may stay in flight
    if (nT - 1 - u >= RING - 2)
      __asm__ volatile("s_waitcnt vmcnt(%0)" ::"n"((RING - 2) * kBbLoads) : "memory");
    else
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    const u32x4 *sb = &sbuf[rb * kBufChunks];
    u32x4 ah[2], al[2], bh[2], bl[2];
    if (live) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int c = h * 64 + 32 * q + li;
        ah[q] = sb[(0 + ti) * kSlotChunks + c];
        al[q] = sb[(2 + ti) * kSlotChunks + c];
        bh[q] = sb[(4 + tj) * kSlotChunks + c];
        bl[q] = sb[(6 + tj) * kSlotChunks + c];
      }
    }
    if (u + RING - 1 < nT) load_stage(u + RING - 1, wb);
    rb = rb == RING - 1 ? 0 : rb + 1;
    wb = wb == RING - 1 ? 0 : wb + 1;
    if (live) {
      bf16x8 Bhi[2], Bli[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Bhi[q] = as_bf16x8(im_operand(bh[q]));
        Bli[q] = as_bf16x8(im_operand(bl[q]));
      }
#pragma unroll
      for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj) {
          floatx16 &R = acc[qi][qj][0], &Im = acc[qi][qj][1];
          const bf16x8 Ah = as_bf16x8(ah[qi]), Al = as_bf16x8(al[qi]);
          const bf16x8 Bh = as_bf16x8(bh[qj]), Bl = as_bf16x8(bl[qj]);
          R = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, R, 0, 0, 0);
          Im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bhi[qj], Im, 0, 0, 0);
          R = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, R, 0, 0, 0);
          Im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bli[qj], Im, 0, 0, 0);
          R = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, R, 0, 0, 0);
          Im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bhi[qj], Im, 0, 0, 0);
        }
    }
  }
  if (!live) return;
  const size_t tile_index = static_cast<size_t>(I) * nb - static_cast<size_t>(I) * (I - 1) / 2 + (J - I);
  float2 *Ht = H + tile_index * (kTile * kTile);
#pragma unroll
  for (int qi = 0; qi < 2; ++qi)
#pragma unroll
    for (int qj = 0; qj < 2; ++qj) {
      float2 hv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * qi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        hv[r] = Ht[row * kTile + 32 * qj + li];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * qi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = 32 * qj + li;
        hv[r].x += acc[qi][qj][0][r];
        hv[r].y += acc[qi][qj][1][r];
        if (I == J && row == col) hv[r].y = 0.f;
        Ht[row * kTile + col] = hv[r];
      }
    }
}


// Dense N x N copy of the packed Hermitian H (inspection only).
__global__ __launch_bounds__(256) void k_gram_dense(int N, int nb, const float2 *__restrict__ H,
                                                    const int *__restrict__ tile_row0,
                                                    float2 *__restrict__ out) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= static_cast<size_t>(N) * N) return;
  const int i = static_cast<int>(idx / N), j = static_cast<int>(idx % N);
  const int I = i / kTile, J = j / kTile;
  float2 v;
  if (I <= J) {
    v = H[static_cast<size_t>(tile_row0[I] + (J - I)) * kTile * kTile + (i % kTile) * kTile + (j % kTile)];
  } else {
    const float2 u = H[static_cast<size_t>(tile_row0[J] + (I - J)) * kTile * kTile + (j % kTile) * kTile + (i % kTile)];
    v = make_float2(u.x, -u.y);
  }
  out[idx] = v;
}

// Sampled entries H[i_n, j_n] of the packed Hermitian H (inspection only).
__global__ __launch_bounds__(256) void k_gram_entries(int n, int N, const float2 *__restrict__ H,
                                                      const int *__restrict__ tile_row0,
                                                      const int *__restrict__ ii,
                                                      const int *__restrict__ jj,
                                                      float2 *__restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int i = ii[t], j = jj[t];
  if (i < 0 || j < 0 || i >= N || j >= N) {
    out[t] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    return;
  }
  const int I = i / kTile, J = j / kTile;
  if (I <= J) {
    out[t] = H[static_cast<size_t>(tile_row0[I] + (J - I)) * kTile * kTile + (i % kTile) * kTile + (j % kTile)];
  } else {
    const float2 u = H[static_cast<size_t>(tile_row0[J] + (I - J)) * kTile * kTile + (j % kTile) * kTile + (i % kTile)];
    out[t] = make_float2(u.x, -u.y);
  }
}

}  // namespace

// Three-product form: 25% fewer MFMA instructions, measured 164 -> 124 us at
// N = 4096 and 4.41 -> 3.30 ms at N = 16384; max |H - FP64| on sampled entries
// 2.0e-4 vs 2.8e-4 (N = 4096, K = 256) and 7.3e-4 vs 1.0e-3 (N = 16384, K = 512).
constexpr bool kGramThree = true;

hipError_t launch_gram_fp32(const Geom &g, const float2 *A, float2 *H,
                            const int2 *tile_ij, int ntiles_grid, const CorrArgs &corr,
                            const GramSplit &split, int kb, const ScalarArgs *sc, bool *sc_done,
                            hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (sc_done) *sc_done = false;
  if (g.K > kMaxFreq || ntiles_grid % 8 != 0 || (kb != 16 && kb != 32)) return hipErrorInvalidValue;
  const bool fix = split.nsplit > 0;
  if (fix && (split.parts < 2 || split.parts > (g.K + kb - 1) / kb ||
              split.parts > kGramSplitMaxParts || !split.P || !split.ij))
    return hipErrorInvalidValue;
  // the events bracket both launches, so a timed Gram update includes the fix-up
  auto kern = kb == 32 ? k_gram_fp32<32, kGramThree> : k_gram_fp32<16, kGramThree>;
  if (t0)
    hipExtLaunchKernelGGL(kern, dim3(ntiles_grid), dim3(256), 0, st, t0, fix ? nullptr : t1, 0, g.K,
                          g.Npad, ntiles_grid, A, tile_ij, H, corr, split.P, split.parts);
  else
    hipLaunchKernelGGL(kern, dim3(ntiles_grid), dim3(256), 0, st, g.K, g.Npad, ntiles_grid, A,
                       tile_ij, H, corr, split.P, split.parts);
  if (fix) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool scal = sc != nullptr;
    const ScalarArgs sa = scal ? *sc : ScalarArgs{};
    const dim3 grid(split.nsplit + (scal ? 1 : 0), kTile * kTile / 256);
    auto fk = scal ? k_gram_fixup<true> : k_gram_fixup<false>;
    if (t0)
      hipExtLaunchKernelGGL(fk, grid, dim3(256), 0, st, nullptr, t1, 0, g.Npad / kTile, split.parts,
                            split.ij, static_cast<const float2 *>(split.P), H, sa);
    else
      hipLaunchKernelGGL(fk, grid, dim3(256), 0, st, g.Npad / kTile, split.parts, split.ij,
                         static_cast<const float2 *>(split.P), H, sa);
    if (scal && sc_done) *sc_done = true;
  }
  return hipGetLastError();
}

hipError_t launch_corr(const Geom &g, const float2 *A, const float2 *d,
                       double cos_c, double sin_c, float2 *b, DevScalars *scal,
                       int first, hipStream_t st, float2 *delta) {
  const size_t lds = static_cast<size_t>(g.K) * sizeof(float2);
  hipLaunchKernelGGL(k_corr, dim3(g.Npad / kCorrPix), dim3(256), lds, st, g, A, d,
                     static_cast<float>(cos_c), static_cast<float>(sin_c), b, scal, first, delta);
  return hipGetLastError();
}

hipError_t launch_gram_bf16x3(const Geom &g, const float2 *A, unsigned *Ahi, unsigned *Alo,
                              float2 *H, const int2 *tile_ij, int ntiles_grid, const int2 *blocks,
                              int nblocks, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (g.K % kBfKB != 0) return hipErrorInvalidValue;
  dim3 sgrid(g.Npad / kSplitTile, (g.K + kSplitTile - 1) / kSplitTile);
  hipLaunchKernelGGL(k_split_bf16, sgrid, dim3(256), 0, st, g.K, g.Npad, A, Ahi, Alo);
  if (blocks) {  // 2 x 2 tile blocks, one 64 x 64 tile per wave
    if (t0)
      hipExtLaunchKernelGGL(k_gram_bf16_blk<kBbRing>, dim3(nblocks), dim3(256), 0, st, t0, t1, 0, g.K, g.Npad,
                            static_cast<const unsigned *>(Ahi), static_cast<const unsigned *>(Alo),
                            blocks, H);
    else
      hipLaunchKernelGGL(k_gram_bf16_blk<kBbRing>, dim3(nblocks), dim3(256), 0, st, g.K, g.Npad,
                         static_cast<const unsigned *>(Ahi), static_cast<const unsigned *>(Alo),
                         blocks, H);
    return hipGetLastError();
  }
  if (t0)  // the events time the product kernel only
    hipExtLaunchKernelGGL(k_gram_bf16x3, dim3(ntiles_grid), dim3(256), 0, st, t0, t1, 0, g.K,
                          g.Npad, ntiles_grid, static_cast<const unsigned *>(Ahi),
                          static_cast<const unsigned *>(Alo), tile_ij, H);
  else
    hipLaunchKernelGGL(k_gram_bf16x3, dim3(ntiles_grid), dim3(256), 0, st, g.K, g.Npad, ntiles_grid,
                       Ahi, Alo, tile_ij, H);
  return hipGetLastError();
}

hipError_t launch_gram_entries(const Geom &g, const float2 *H, const int *tile_row0, int n,
                               const int *ii, const int *jj, float2 *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_entries, dim3((n + 255) / 256), dim3(256), 0, st, n, g.N, H, tile_row0,
                     ii, jj, out);
  return hipGetLastError();
}

hipError_t launch_gram_dense(const Geom &g, const float2 *H,
                             const int *tile_row0, float2 *out,
                             hipStream_t st) {
  const size_t n = static_cast<size_t>(g.N) * g.N;
  hipLaunchKernelGGL(k_gram_dense, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                     g.N, g.Npad / kTile, H, tile_row0, out);
  return hipGetLastError();
}

}  // namespace ofista
