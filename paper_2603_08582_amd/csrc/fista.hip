// One step of Algorithm 1 (Online FISTA, inner loop) as a single launch:
//   y = H z, g = y - b, u = z - tau g, c = S_{lambda tau}(u),
//   z' = c + beta (c - c_prev)
// fused with one power-iteration step on the same pass over H:
//   y_w = H w, rho parts Re<w, y_w>, w' = y_w / |w|.
//
// H is stored as packed upper tiles, so each tile (I, J), I < J, serves two
// products: y_I += H_IJ z_J (rows) and y_J += H_IJ^H z_I (columns).  This is
// the memory-bound kernel of the path: every element of the upper triangle is
// read exactly once per step (8 bytes for 16 FP32 FMAs).
//
// Work item = tile row I and a run of up to 2 (or 4) tiles J0..J1-1.  Wave w
// of the 256-thread workgroup owns rows 16w..16w+15 of each tile and lane l
// owns column l, so row partial sums stay in registers across the run and are
// reduced across lanes once per item; column partials are reduced across the
// 4 waves through LDS.  Every partial lands in its own slot (slot_index) --
// no floating-point atomics, so the result is bitwise deterministic.
//
// A step is two launches: the tile pass (k_step_tiles) writes the slots, and
// k_step_update (one workgroup per tile row) sums each row's slots in fixed
// order and applies the shrink / momentum / power update.  Stream order makes
// the slots visible to the update.  (Fusing the update into the tile pass with
// an arrival counter needs every workgroup to wait for its slot stores and the
// counter round trip before it can retire; on gfx950 that idle time doubled
// the step even with coherent stores instead of cache-wide fences.)
#include "ofista_internal.h"

namespace ofista {
namespace {

__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 x) {
  // acc + a * x
  acc.x = fmaf(a.x, x.x, acc.x);
  acc.x = fmaf(-a.y, x.y, acc.x);
  acc.y = fmaf(a.x, x.y, acc.y);
  acc.y = fmaf(a.y, x.x, acc.y);
  return acc;
}

__device__ __forceinline__ float2 cmac_conj(float2 acc, float2 a, float2 x) {
  // acc + conj(a) * x
  acc.x = fmaf(a.x, x.x, acc.x);
  acc.x = fmaf(a.y, x.y, acc.x);
  acc.y = fmaf(a.x, x.y, acc.y);
  acc.y = fmaf(-a.y, x.x, acc.y);
  return acc;
}

constexpr int kRowsPerWave = kTile / 4;  // 16

// Fixed-order tree sum of one double per thread over the 256-thread block.
__device__ double block_sum256(double v, double *red) {
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

// Fixed-order sum over a wave (every lane ends with its own, lane 0 with the
// canonical tree).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Update: kUpdSplit workgroups per tile row, each owning kUpdRows rows.
// Thread (part p, row r) adds the valid slots v = p, p + kUpdParts, ... of its
// row; slots are read kUpdBatch at a time (index clamped in range, unused
// values replaced by zero after the load), then the parts are summed in LDS
// in increasing p.
constexpr int kUpdRows = kTile / kUpdSplit;  // 16
constexpr int kUpdParts = 256 / kUpdRows;    // 16
constexpr int kUpdBatch = 4;

// The per-row arithmetic of the update (gradient step, shrink, momentum,
// power vector and its two inner-product parts), with every fused
// multiply-add written out so that each kernel running it rounds alike.
struct RowUpdate {
  float2 u, c, z, w;
  double r, m;  // Re<w, H w> and |w'|^2 parts of this row
};
__device__ __forceinline__ RowUpdate row_update(float4 s, float2 z, float2 cold, float2 bi,
                                                float2 w, float tau, float alpha, float beta,
                                                float inv_wn) {
  RowUpdate o;
  const float gx = s.x - bi.x, gy = s.y - bi.y;
  o.u = make_float2(fmaf(-tau, gx, z.x), fmaf(-tau, gy, z.y));
  const float mag = sqrtf(fmaf(o.u.x, o.u.x, o.u.y * o.u.y));
  float cx = 0.f, cy = 0.f;
  if (mag > alpha) {
    const float f = 1.f - alpha / mag;
    cx = o.u.x * f;
    cy = o.u.y * f;
  }
  o.c = make_float2(cx, cy);
  o.z = make_float2(fmaf(beta, cx - cold.x, cx), fmaf(beta, cy - cold.y, cy));
  o.w = make_float2(s.z * inv_wn, s.w * inv_wn);
  o.r = fma(static_cast<double>(w.x), static_cast<double>(s.z),
            static_cast<double>(w.y) * static_cast<double>(s.w));
  o.m = fma(static_cast<double>(o.w.x), static_cast<double>(o.w.x),
            static_cast<double>(o.w.y) * static_cast<double>(o.w.y));
  return o;
}

// Slot v of target row R: the column partials j < R come first, then the run
// starts j = R, R + chunk, ... (row partials).
__device__ __forceinline__ int valid_slot(int v, int R, int chunk) {
  return v < R ? v : R + (v - R) * chunk;
}

template <bool PARTIALS>
__global__ __launch_bounds__(256) void k_step_update(StepArgs a) {
  __shared__ float4 red[kUpdParts][kUpdRows];
  __shared__ double wred[4];
  const int R = blockIdx.x / kUpdSplit, sub = blockIdx.x % kUpdSplit;
  const int nb = a.nb, chunk = a.chunk, nparts = kUpdSplit * nb;
  const int t = threadIdx.x;
  const int r = t % kUpdRows, part = t / kUpdRows;
  // step and threshold read first: a load after the barrier below would be
  // a round trip of its own at the end of the kernel
  const float tau = static_cast<float>(a.scal->tau);
  const float alpha = static_cast<float>(a.scal->alpha);
  const int i = R * kTile + sub * kUpdRows + r;
  // tile-pass slots: column partials j < R, then the run starts; store-all:
  // the nchunks partial rows of P
  const int nvalid = PARTIALS ? a.nchunks : R + (nb - R + chunk - 1) / chunk;
  const bool live = t < kUpdRows && i < a.N;
  const f32x4 *q = PARTIALS ? reinterpret_cast<const f32x4 *>(a.P + i)
                            : reinterpret_cast<const f32x4 *>(a.Q + (i - R * kTile));
  auto slot_off = [&](int v) {
    const int vc = v < nvalid ? v : nvalid - 1;
    return PARTIALS ? static_cast<size_t>(vc) * a.Npad
                    : slot_index(valid_slot(vc, R, chunk), R, nb) * kTile;
  };
  // Every load of the first round is issued before any value is used (the
  // first batch of slots, the row's vectors, the first |w|^2 part of the
  // vector this step multiplied): one round trip instead of three.  Indices
  // are clamped in range and unused values dropped afterwards (i < Npad for
  // every thread; threads past nvalid or nparts add zeros, as the loops below
  // would have added nothing).
  f32x4 x[kUpdBatch];
#pragma unroll
  for (int u = 0; u < kUpdBatch; ++u) x[u] = __builtin_nontemporal_load(q + slot_off(part + kUpdParts * u));
  const float2 zl = a.zc[i], coldl = a.cc[i], bil = a.b[i], wl = a.wc[i];
  const double m0 = a.slot_prev[nparts + (t < nparts ? t : 0)];
  const float2 zero2 = make_float2(0.f, 0.f);
  const float2 z = live ? zl : zero2, cold = live ? coldl : zero2, bi = live ? bil : zero2,
               w = live ? wl : zero2;
  double m = 0.0;
  if (t < nparts) m += m0;
  for (int j = t + 256; j < nparts; j += 256) m += a.slot_prev[nparts + j];
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int v0 = part;; v0 += kUpdParts * kUpdBatch) {
    if (v0 != part) {
#pragma unroll
      for (int u = 0; u < kUpdBatch; ++u) x[u] = __builtin_nontemporal_load(q + slot_off(v0 + kUpdParts * u));
    }
#pragma unroll
    for (int u = 0; u < kUpdBatch; ++u) {
      const bool ok = v0 + kUpdParts * u < nvalid;
      acc.x += ok ? x[u].x : 0.f;
      acc.y += ok ? x[u].y : 0.f;
      acc.z += ok ? x[u].z : 0.f;
      acc.w += ok ? x[u].w : 0.f;
    }
    if (v0 + kUpdParts * kUpdBatch >= nvalid) break;
  }
  red[part][r] = acc;
  m = wave_sum(m);
  if ((t & 63) == 0) wred[t >> 6] = m;
  __syncthreads();
  if (t >= kUpdRows) return;
  const double wn2 = ((wred[0] + wred[1]) + wred[2]) + wred[3];
  float4 s = red[0][t];
#pragma unroll
  for (int p = 1; p < kUpdParts; ++p) {
    const float4 v = red[p][t];
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  const float inv_wn = static_cast<float>(1.0 / sqrt(wn2));
  double rpart = 0.0, mpart = 0.0;
  if (live) {
    const RowUpdate o = row_update(s, z, cold, bi, w, tau, alpha, a.beta, inv_wn);
    if (a.urec) a.urec[i] = o.u;  // kept for the reverse pass
    a.cn[i] = o.c;
    a.zn[i] = o.z;
    a.wn[i] = o.w;
    rpart = o.r;
    mpart = o.m;
  } else {
    a.cn[i] = make_float2(0.f, 0.f);
    a.zn[i] = make_float2(0.f, 0.f);
    a.wn[i] = make_float2(0.f, 0.f);
  }
  // parts of Re<w, Hw> and |w'|^2 over this workgroup's rows, fixed order
#pragma unroll
  for (int off = kUpdRows / 2; off >= 1; off >>= 1) {
    rpart += __shfl_xor(rpart, off);
    mpart += __shfl_xor(mpart, off);
  }
  if (t == 0) {
    a.slot_cur[blockIdx.x] = rpart;
    a.slot_cur[nparts + blockIdx.x] = mpart;
  }
}

template <int CH, bool CACHED, bool NTSTORE>
__global__ __launch_bounds__(256) void k_step_tiles(StepArgs a) {
  __shared__ float4 colbuf[CH][4][64];

  const WorkItem it = a.items[blockIdx.x];
  const int I = it.I, J0 = it.J0, J1 = it.J1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int row0 = wave * kRowsPerWave;

  // z_I, w_I for this wave's 16 rows (wave-uniform)
  float2 zI[kRowsPerWave], wI[kRowsPerWave];
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    zI[q] = a.zc[I * kTile + row0 + q];
    wI[q] = a.wc[I * kTile + row0 + q];
  }
  float2 ryz[kRowsPerWave], ryw[kRowsPerWave];
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    ryz[q] = make_float2(0.f, 0.f);
    ryw[q] = make_float2(0.f, 0.f);
  }

  const float2 *Hrow = a.H + static_cast<size_t>(it.toff) * (kTile * kTile) + row0 * kTile + lane;
  float2 hA[kRowsPerWave], hB[kRowsPerWave], zA, wA, zB, wB;
  auto issue = [&](float2 (&h)[kRowsPerWave], float2 &zz, float2 &ww, int jj) {
    const int J = min(J0 + jj, J1 - 1);
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      // cached loads when H fits the last-level cache (it stays there from
      // step to step), nontemporal loads when it streams from HBM
      const float2 *ph = Hrow + static_cast<size_t>(J) * kTile * kTile + q * kTile;
      if constexpr (CACHED) {
        h[q] = *ph;
      } else {
        const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(ph));
        h[q] = make_float2(v.x, v.y);
      }
    }
    zz = a.zc[J * kTile + lane];
    ww = a.wc[J * kTile + lane];
  };
  auto multiply = [&](const float2 (&h)[kRowsPerWave], const float2 &zj, const float2 &wj, int jj) {
    float2 cz = make_float2(0.f, 0.f), cw = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      ryz[q] = cmac(ryz[q], h[q], zj);
      ryw[q] = cmac(ryw[q], h[q], wj);
      cz = cmac_conj(cz, h[q], zI[q]);
      cw = cmac_conj(cw, h[q], wI[q]);
    }
    colbuf[jj][wave][lane] = make_float4(cz.x, cz.y, cw.x, cw.y);
  };
  // Two statically named register sets (ping-pong): the loads of tile jj+1
  // are issued before tile jj is multiplied.  Tiles past the end of a short
  // run are clamped to its last tile (a re-read that hits in cache) and not
  // multiplied.  (16-byte loads covering two rows per instruction measured
  // 2x slower here than these 8-byte row loads.)
  const int nrun = J1 - J0;
  issue(hA, zA, wA, 0);
#pragma unroll
  for (int jj = 0; jj < CH; jj += 2) {
    if (jj + 1 < CH) issue(hB, zB, wB, jj + 1);
    if (jj < nrun) multiply(hA, zA, wA, jj);
    if (jj + 2 < CH) issue(hA, zA, wA, jj + 2);
    if (jj + 1 < CH && jj + 1 < nrun) multiply(hB, zB, wB, jj + 1);
  }

  // Row partials: 16 rows x (yz, yw) = 64 floats per lane, summed over the 64
  // lanes by a halving butterfly; afterwards lane l holds element l
  // (row l/4, component l%4).
  float v[64];
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    v[4 * q + 0] = ryz[q].x;
    v[4 * q + 1] = ryz[q].y;
    v[4 * q + 2] = ryw[q].x;
    v[4 * q + 3] = ryw[q].y;
  }
#pragma unroll
  for (int half = 32; half >= 1; half >>= 1) {
    const bool upper = (lane & half) != 0;
#pragma unroll
    for (int e = 0; e < half; ++e) {
      const float send = upper ? v[e] : v[e + half];
      const float keep = upper ? v[e + half] : v[e];
      v[e] = keep + __shfl_xor(send, half);
    }
  }
  // Column partials of the off-diagonal tiles: sum the 4 waves in fixed order.
  // (The row partial is stored after this barrier: a store issued before it
  // would be waited for there.)
  __syncthreads();
#pragma unroll
  for (int jj = threadIdx.x >> 6; jj < CH; jj += 4) {
    const int J = J0 + jj;
    if (J < J1 && J != I) {
      float4 s = colbuf[jj][0][lane];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const float4 t = colbuf[jj][w][lane];
        s.x += t.x;
        s.y += t.y;
        s.z += t.z;
        s.w += t.w;
      }
      // column slots are written source-major (scattered target-major stores
      // into the saturated read stream took 3.5% longer at N = 16384)
      float4 *dst = a.Q + slot_index(I, J, a.nb) * kTile + lane;
      if constexpr (NTSTORE)
        __builtin_nontemporal_store(f32x4{s.x, s.y, s.z, s.w}, reinterpret_cast<f32x4 *>(dst));
      else
        *dst = s;
    }
  }
  float *rdst = reinterpret_cast<float *>(a.Q + slot_index(J0, I, a.nb) * kTile + row0) + lane;
  if constexpr (NTSTORE)
    __builtin_nontemporal_store(v[0], rdst);
  else
    *rdst = v[0];
}

// ---------------------------------------------------------------------------
// Resident steps: every FISTA step of one reconstruct call in a single
// cooperative launch of one 512-thread workgroup per CU.  A step is the same
// two phases as the launch pair above -- the tile pass writing the slots, then
// the update summing them -- with a grid barrier after each phase instead of a
// kernel boundary.  Workgroup g owns work items g, g + G, g + 2G, ... (G =
// workgroups, at most kResMaxItems items) for the whole call, in rounds of
// two: in round r its two groups of 4 waves each take item 2r + (group).  The
// tiles of round 0 are copied into LDS once, those of round 1 into the
// registers of their group, and round 2 (the single-tile runs some
// workgroups get) reads H from memory; update block 2g + (group), +2G, ...
// follows.  The arithmetic of an item and of an update block is that of
// k_step_tiles<2> / k_step_update<false> with the same summation orders, so
// the iterates are bitwise those of the launch pair.  At N = 4096 on 256 CUs
// a step measured 26 us (rounds 5.0 + 4.5 + 6.4, update 2.6, two barriers and
// the z, w staging about 6) against 17.6 us for the launch pair, so it is an
// option, not the default.
//
// Values that cross workgroups within the launch (slots, z, c, w, the power
// parts) are written and read with agent-scope atomic stores and loads
// (global_store / global_load with sc1): they bypass the non-coherent L1 and
// the scalar cache, and reach the coherence point across the XCDs' L2s.  The
// grid barrier: each workgroup waits for its own stores (the fence of
// __syncthreads), adds 1 to the counter of its XCD group (workgroup g on
// counter g % 8, so 32 arrivals per counter instead of 256 on one address),
// and lanes 0..7 of the first wave poll the 8 counters until each holds its
// workgroup count times the barrier generation.  Polls are bounded: past the
// limit the workgroup records a fault in the scalars and stops waiting at
// later barriers, so a launch that could not be co-resident ends instead of
// hanging (its results are then invalid and the next state query reports the
// fault).
constexpr unsigned kBarSpinLimit = 1u << 20;  // polls (each ~1 us): about a second

__device__ __forceinline__ float2 ld_agent2(const float2 *p) {
  const unsigned long long v =
      __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float2 *>(p)),
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float2, v);
}
__device__ __forceinline__ void st_agent2(float2 *p, float2 v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ f32x4 ld_agent4(const float4 *p) {
  const float2 lo = ld_agent2(reinterpret_cast<const float2 *>(p));
  const float2 hi = ld_agent2(reinterpret_cast<const float2 *>(p) + 1);
  return f32x4{lo.x, lo.y, hi.x, hi.y};
}
__device__ __forceinline__ void st_agent4(float4 *p, float4 v) {
  st_agent2(reinterpret_cast<float2 *>(p), make_float2(v.x, v.y));
  st_agent2(reinterpret_cast<float2 *>(p) + 1, make_float2(v.z, v.w));
}
__device__ __forceinline__ double ld_agent_d(const double *p) {
  const unsigned long long v =
      __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ void st_agent_d(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_f(float *p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned *>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false once a wait has timed out; the caller then passes
// broken = true to the later barriers, which no longer wait.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned gen, DevScalars *scal,
                                             bool broken) {
  __syncthreads();  // this workgroup's stores have completed
  __shared__ unsigned timed_out;
  if (threadIdx.x == 0) timed_out = 0;
  __syncthreads();
  if (threadIdx.x < 8) {
    const unsigned nwg = gridDim.x;
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&bar[(blockIdx.x & 7) * kBarStride], 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    const unsigned x = threadIdx.x;
    const unsigned target = (nwg > x ? (nwg - x + 7) / 8 : 0) * gen;
    unsigned spins = 0;
    while (!broken && __hip_atomic_load(&bar[x * kBarStride], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kBarSpinLimit) {
        __hip_atomic_store(&scal->fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        timed_out = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return !broken && timed_out == 0;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses,
// not for its global stores (the fence of __syncthreads would wait for
// those, a round trip to the coherence point per item).
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// One work item of the tile pass (tile row I, run J0..J1-1 of at most 2 tiles)
// with its H elements from hfetch(jj, q) (row row0 + q, column lane of tile
// J0 + jj) and z, w of row blocks I, J0, J0 + 1 from the LDS staging zs, ws
// ([0]: block I, [1 + jj]: block J0 + jj): the multiplies, reductions and slot
// stores of k_step_tiles<2>.
template <typename HFetch>
__device__ __forceinline__ void resident_item(const WorkItem it, int nb, int wave,
                                              const float2 (*zs)[kTile],
                                              const float2 (*ws)[kTile], float4 *Q,
                                              float4 (*colbuf)[4][64], bool mine, HFetch hfetch) {
  // a group without an item this round still meets the workgroup barrier
  const int I = it.I, J0 = it.J0, J1 = it.J1;
  const int lane = threadIdx.x & 63;
  const int row0 = wave * kRowsPerWave;
  const int nrun = J1 - J0;
  float v[64];
  if (mine) {
    float2 zj[2], wj[2];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      zj[jj] = zs[1 + jj][lane];
      wj[jj] = ws[1 + jj][lane];
    }
    float2 ryz[kRowsPerWave], ryw[kRowsPerWave];
    float2 cz[2], cw[2];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) cz[jj] = cw[jj] = make_float2(0.f, 0.f);
    // rows in the outer loop: each accumulator sees the same sequence of
    // operations as in k_step_tiles (ryz[q] over jj = 0, 1; cz[jj] over q)
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      const float2 zI = zs[0][row0 + q];
      const float2 wI = ws[0][row0 + q];
      ryz[q] = ryw[q] = make_float2(0.f, 0.f);
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        if (jj < nrun) {
          const float2 h = hfetch(jj, q);
          ryz[q] = cmac(ryz[q], h, zj[jj]);
          ryw[q] = cmac(ryw[q], h, wj[jj]);
          cz[jj] = cmac_conj(cz[jj], h, zI);
          cw[jj] = cmac_conj(cw[jj], h, wI);
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
      if (jj < nrun) colbuf[jj][wave][lane] = make_float4(cz[jj].x, cz[jj].y, cw[jj].x, cw[jj].y);
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      v[4 * q + 0] = ryz[q].x;
      v[4 * q + 1] = ryz[q].y;
      v[4 * q + 2] = ryw[q].x;
      v[4 * q + 3] = ryw[q].y;
    }
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
      const bool upper = (lane & half) != 0;
#pragma unroll
      for (int e = 0; e < half; ++e) {
        const float send = upper ? v[e] : v[e + half];
        const float keep = upper ? v[e + half] : v[e];
        v[e] = keep + __shfl_xor(send, half);
      }
    }
  }
  lds_barrier();
  if (mine) {
    if (wave < 2) {
      const int jj = wave;
      const int J = J0 + jj;
      if (J < J1 && J != I) {
        float4 s = colbuf[jj][0][lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
          const float4 t = colbuf[jj][w][lane];
          s.x += t.x;
          s.y += t.y;
          s.z += t.z;
          s.w += t.w;
        }
        st_agent4(Q + slot_index(I, J, nb) * kTile + lane, s);
      }
    }
    st_agent_f(reinterpret_cast<float *>(Q + slot_index(J0, I, nb) * kTile + row0) + lane, v[0]);
  }
}

static_assert(kChunk == 2, "resident items are runs of at most two tiles");

__global__ __launch_bounds__(512) void k_steps_resident(ResidentArgs a) {
  __shared__ float2 htile[2 * kResLdsItems][kTile * kTile];  // 128 KB
  // the column buffers of the two item groups (tile pass) share their space
  // with the update's reduction buffers
  __shared__ float4 scratch_lds[2 * 2 * 4 * 64];
  float4 (*colbuf)[2][4][64] = reinterpret_cast<float4 (*)[2][4][64]>(scratch_lds);
  float4 (*red)[kUpdRows] = reinterpret_cast<float4 (*)[kUpdRows]>(scratch_lds);
  static_assert(2 * kUpdParts * kUpdRows <= 2 * 2 * 4 * 64, "update buffers fit the column buffers");
  __shared__ double wred[2][4];
  // z and w of row blocks I, J0, J0 + 1 of every item, staged once per step
  __shared__ float2 zst[kResMaxItems][3][kTile], wst[kResMaxItems][3][kTile];
  __shared__ int blk[kResMaxItems][3];   // row blocks staged per item
  __shared__ int itab[kResMaxItems][4];  // I, J0, J1, first tile index - I
  const int G = gridDim.x, g = blockIdx.x;
  // two groups of 4 waves; group grp works on items grp, grp + 2, grp + 4 of
  // this workgroup, wave wig of the group on rows 16 wig ..
  const int wave8 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = wave8 >> 2, wig = wave8 & 3;
  const int lane = threadIdx.x & 63;
  const int row0 = wig * kRowsPerWave;
  const int nb = a.nb, nparts = a.nparts;
  const int nmine = g < a.nitems ? min((a.nitems - g + G - 1) / G, kResMaxItems) : 0;
  // this workgroup's items and their first tile indices, read once into
  // LDS: a table load between the agent-scope stores of the steps would be a
  // vector load whose wait drains those stores
  if (threadIdx.x < kResMaxItems) {
    const int m = threadIdx.x;
    const WorkItem it = m < nmine ? a.items[g + m * G] : WorkItem{0, 0, 1, 0};
    itab[m][0] = it.I;
    itab[m][1] = it.J0;
    itab[m][2] = it.J1;
    itab[m][3] = it.toff;
    blk[m][0] = it.I;
    blk[m][1] = it.J0;
    blk[m][2] = min(it.J0 + 1, it.J1 - 1);
  }
  __syncthreads();
  auto item = [&](int m) {
    return WorkItem{__builtin_amdgcn_readfirstlane(itab[m][0]),
                    __builtin_amdgcn_readfirstlane(itab[m][1]),
                    __builtin_amdgcn_readfirstlane(itab[m][2]), 0};
  };
  auto tile0 = [&](int m) {
    return static_cast<size_t>(__builtin_amdgcn_readfirstlane(itab[m][3])) * (kTile * kTile);
  };
  // items 0, 1 (round 0) keep their tiles in LDS, items 2, 3 (round 1) in the
  // registers of their group, item 4 (round 2) reads them from memory.  Each
  // thread copies, and later reads back, only its own elements (rows row0..,
  // column lane of its group's item).
  float2 hreg[2][kRowsPerWave];
  {
    const int m = kResLdsItems + grp;
    if (m < nmine) {
      const WorkItem it = item(m);
      const float2 *Hrow = a.H + tile0(m) + row0 * kTile + lane;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int J = min(it.J0 + jj, it.J1 - 1);
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q)
          hreg[jj][q] = Hrow[static_cast<size_t>(J) * kTile * kTile + q * kTile];
      }
    }
  }
  if (grp < nmine) {
    const int m = grp;
    const WorkItem it = item(m);
    const float2 *Hrow = a.H + tile0(m) + row0 * kTile + lane;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int J = min(it.J0 + jj, it.J1 - 1);
#pragma unroll
      for (int q = 0; q < kRowsPerWave; ++q)
        htile[2 * m + jj][(row0 + q) * kTile + lane] =
            Hrow[static_cast<size_t>(J) * kTile * kTile + q * kTile];
    }
  }
  const float tau = static_cast<float>(a.scal->tau);
  const float alpha = static_cast<float>(a.scal->alpha);
  unsigned gen = a.bar_gen;
  bool broken = false;
  for (int k = 0; k < a.iters; ++k) {
    const int p = (a.p0 + k) & 1;
    const float2 *zc = (k == 0 && a.warm) ? a.cbuf[p] : a.zbuf[p];
    const float2 *wc = a.wbuf[p], *cc = a.cbuf[p];
    float2 *cn = a.cbuf[p ^ 1], *zn = a.zbuf[p ^ 1], *wn = a.wbuf[p ^ 1];
    const double *slot_prev = a.slots[p];
    double *slot_cur = a.slots[p ^ 1];
    // stage z, w of the items' row blocks: every load issued before any is
    // used (agent-scope loads keep their program order)
    {
      constexpr int kPer = (kResMaxItems * 3 * kTile + 511) / 512;
      const int n = nmine * 3 * kTile;
      float2 zv[kPer], wv[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 512 * u;
        if (e < n) {
          const int B = blk[e / (3 * kTile)][(e / kTile) % 3];
          zv[u] = ld_agent2(zc + B * kTile + (e % kTile));
          wv[u] = ld_agent2(wc + B * kTile + (e % kTile));
        }
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 512 * u;
        if (e < n) {
          (&zst[0][0][0])[e] = zv[u];
          (&wst[0][0][0])[e] = wv[u];
        }
      }
      __syncthreads();
    }
    // tile pass: round r, group grp takes item 2 r + grp; both groups meet
    // at the workgroup barriers of every round (colbuf per group)
#pragma unroll
    for (int r = 0; r < (kResMaxItems + 1) / 2; ++r) {
      if (2 * r >= nmine) break;
      const int m = 2 * r + grp;
      const bool mine = m < nmine;
      const int mc = mine ? m : 2 * r;  // a valid index for the idle group
      const WorkItem it = item(mc);
      const size_t tb = tile0(mc);
      if (r == 0) {
        const float2 *ht = &htile[2 * grp][0];
        resident_item(it, nb, wig, zst[mc], wst[mc], a.Q, colbuf[grp], mine,
                      [&](int jj, int q) { return ht[jj * kTile * kTile + (row0 + q) * kTile + lane]; });
      } else if (r == 1) {
        resident_item(it, nb, wig, zst[mc], wst[mc], a.Q, colbuf[grp], mine,
                      [&](int jj, int q) { return hreg[jj][q]; });
      } else {
        // (round 2 holds the single-tile runs of a few workgroups: H read in
        // the multiply loop, no buffer beside the resident registers)
        const float2 *Hrow = a.H + tb + row0 * kTile + lane;
        resident_item(it, nb, wig, zst[mc], wst[mc], a.Q, colbuf[grp], mine, [&](int jj, int q) {
          return Hrow[static_cast<size_t>(min(it.J0 + jj, it.J1 - 1)) * kTile * kTile + q * kTile];
        });
      }
      lds_barrier();  // colbuf is reused in the next round
    }
    broken = !grid_barrier(a.bar, ++gen, a.scal, broken);
    // update (k_step_update<false> per block)
    const float beta = a.beta[k];
    // group grp runs update block 2 g + grp (+ 2G, ...); both groups meet at
    // the workgroup barriers
    for (int ub0 = 2 * g; ub0 < kUpdSplit * nb; ub0 += 2 * G) {
      const int ub = ub0 + grp;
      const bool active = ub < kUpdSplit * nb;
      const int ubc = active ? ub : ub0;
      const int R = ubc / kUpdSplit, sub = ubc % kUpdSplit;
      const int t = threadIdx.x & 255;
      const int r = t % kUpdRows, part = t / kUpdRows;
      const int i = R * kTile + sub * kUpdRows + r;
      const int nvalid = R + (nb - R + kChunk - 1) / kChunk;
      const bool live = active && t < kUpdRows && i < a.N;
      // every load of the block is issued before any is used (agent-scope
      // loads keep their program order): the first batch of slots, the row's
      // vectors, the power parts
      const float4 *q = a.Q + (i - R * kTile);
      f32x4 x[kUpdBatch];
#pragma unroll
      for (int u = 0; u < kUpdBatch; ++u) {
        const int v = part + kUpdParts * u;
        const int vc = v < nvalid ? v : nvalid - 1;
        x[u] = active ? ld_agent4(q + slot_index(valid_slot(vc, R, kChunk), R, nb) * kTile)
                      : f32x4{0.f, 0.f, 0.f, 0.f};
      }
      float2 z = make_float2(0.f, 0.f), cold = z, bi = z, w = z;
      if (live) {
        z = ld_agent2(zc + i);
        cold = ld_agent2(cc + i);
        bi = a.b[i];
        w = ld_agent2(wc + i);
      }
      double mparts[(kResMaxParts + 255) / 256];
#pragma unroll
      for (int u = 0; u < (kResMaxParts + 255) / 256; ++u) {
        const int j = t + 256 * u;
        mparts[u] = active && j < nparts ? ld_agent_d(slot_prev + nparts + j) : 0.0;
      }
      double mm = 0.0;
#pragma unroll
      for (int u = 0; u < (kResMaxParts + 255) / 256; ++u)
        if (t + 256 * u < nparts) mm += mparts[u];
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int v0 = part; active && v0 < nvalid; v0 += kUpdParts * kUpdBatch) {
        if (v0 != part) {
#pragma unroll
          for (int u = 0; u < kUpdBatch; ++u) {
            const int v = v0 + kUpdParts * u;
            const int vc = v < nvalid ? v : nvalid - 1;
            x[u] = ld_agent4(q + slot_index(valid_slot(vc, R, kChunk), R, nb) * kTile);
          }
        }
#pragma unroll
        for (int u = 0; u < kUpdBatch; ++u) {
          const bool ok = v0 + kUpdParts * u < nvalid;
          acc.x += ok ? x[u].x : 0.f;
          acc.y += ok ? x[u].y : 0.f;
          acc.z += ok ? x[u].z : 0.f;
          acc.w += ok ? x[u].w : 0.f;
        }
      }
      red[grp * kUpdParts + part][r] = acc;
      mm = wave_sum(mm);
      if ((t & 63) == 0) wred[grp][t >> 6] = mm;
      __syncthreads();
      if (active && t < kUpdRows) {
        const double wn2 = ((wred[grp][0] + wred[grp][1]) + wred[grp][2]) + wred[grp][3];
        float4 s = red[grp * kUpdParts][t];
#pragma unroll
        for (int pp = 1; pp < kUpdParts; ++pp) {
          const float4 vv = red[grp * kUpdParts + pp][t];
          s.x += vv.x;
          s.y += vv.y;
          s.z += vv.z;
          s.w += vv.w;
        }
        const float inv_wn = static_cast<float>(1.0 / sqrt(wn2));
        double rpart = 0.0, mpart = 0.0;
        if (live) {
          const RowUpdate o = row_update(s, z, cold, bi, w, tau, alpha, beta, inv_wn);
          st_agent2(cn + i, o.c);
          st_agent2(zn + i, o.z);
          st_agent2(wn + i, o.w);
          rpart = o.r;
          mpart = o.m;
        } else {
          st_agent2(cn + i, make_float2(0.f, 0.f));
          st_agent2(zn + i, make_float2(0.f, 0.f));
          st_agent2(wn + i, make_float2(0.f, 0.f));
        }
#pragma unroll
        for (int off = kUpdRows / 2; off >= 1; off >>= 1) {
          rpart += __shfl_xor(rpart, off);
          mpart += __shfl_xor(mpart, off);
        }
        if (t == 0) {
          st_agent_d(slot_cur + ub, rpart);
          st_agent_d(slot_cur + nparts + ub, mpart);
        }
      }
      __syncthreads();  // red / wred are reused by the next block
    }
    broken = !grid_barrier(a.bar, ++gen, a.scal, broken);
  }
}

// Per-pulse scalars as their own launch (one 256-thread workgroup).
__global__ __launch_bounds__(256) void k_scalars(ScalarArgs a) {
  __shared__ double red[256];
  pulse_scalars(a, red);
}

__global__ void k_fill(unsigned *p, size_t n, unsigned value) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = value;
}

// w_0 = 1/sqrt(N) on the real pixels; slot0 says |w_0|^2 = 1.
__global__ void k_init_power(float2 *w, double *slot0, double *slot1, int N, int Npad, int nparts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Npad) w[i] = make_float2(i < N ? static_cast<float>(1.0 / sqrt(static_cast<double>(N))) : 0.f, 0.f);
  if (i < 2 * nparts) {
    slot0[i] = (i == nparts) ? 1.0 : 0.0;
    slot1[i] = 0.0;
  }
}

// Large-coefficient count: integer atomics, so the result is exact whatever
// the order.
__global__ __launch_bounds__(256) void k_count_large(const float2 *__restrict__ c, int M, float thr,
                                                     unsigned *__restrict__ count) {
  unsigned n = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
    const float2 v = c[i];
    n += sqrtf(v.x * v.x + v.y * v.y) > thr ? 1u : 0u;
  }
  __shared__ unsigned red[256];
  red[threadIdx.x] = n;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0]) atomicAdd(count, red[0]);
}

// ---------------------------------------------------------------------------
// Store-all comparator (Section III-D): gradient from the stored pulses,
// two passes over the stacked operator per step.

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per stacked row r: U[r] = (G_r z - D_r, G_r w), lanes striding
// over the coefficients (coalesced rows), fixed-order wave sums.
__global__ __launch_bounds__(256) void k_store_forward(const float2 *__restrict__ G,
                                                       const float2 *__restrict__ D, int rows,
                                                       int Npad, int M,
                                                       const float2 *__restrict__ z,
                                                       const float2 *__restrict__ w,
                                                       float4 *__restrict__ U) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;  // whole waves
  const float2 *g = G + static_cast<size_t>(r) * Npad;
  float zr = 0.f, zi = 0.f, wr = 0.f, wi = 0.f;
  for (int m = lane; m < M; m += 64) {
    const float2 a = g[m], x = z[m], y = w[m];
    zr = fmaf(a.x, x.x, fmaf(-a.y, x.y, zr));
    zi = fmaf(a.x, x.y, fmaf(a.y, x.x, zi));
    wr = fmaf(a.x, y.x, fmaf(-a.y, y.y, wr));
    wi = fmaf(a.x, y.y, fmaf(a.y, y.x, wi));
  }
  zr = wave_sum_f32(zr);
  zi = wave_sum_f32(zi);
  wr = wave_sum_f32(wr);
  wi = wave_sum_f32(wi);
  if (lane == 0) {
    const float2 d = D[r];
    U[r] = make_float4(zr - d.x, zi - d.y, wr, wi);
  }
}

// P[c][m] = sum over the rows of chunk c of conj(G[r, m]) (U_z[r], U_w[r]),
// rows in increasing order; thread per coefficient (coalesced rows).
__global__ __launch_bounds__(256) void k_store_adjoint(const float2 *__restrict__ G, int rows,
                                                       int Npad, const float4 *__restrict__ U,
                                                       float4 *__restrict__ P) {
  __shared__ float4 us[kStoreRows];
  const int c = blockIdx.y;
  const int r0 = c * kStoreRows;
  const int rn = min(kStoreRows, rows - r0);
  if (threadIdx.x < kStoreRows)
    us[threadIdx.x] = threadIdx.x < rn ? U[r0 + threadIdx.x] : make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= Npad) return;
  const float2 *g = G + static_cast<size_t>(r0) * Npad + m;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 16
  for (int q = 0; q < rn; ++q) {
    const float2 a = g[static_cast<size_t>(q) * Npad];
    const float4 u = us[q];
    // conj(a) * (u.x + i u.y), conj(a) * (u.z + i u.w)
    acc.x = fmaf(a.x, u.x, fmaf(a.y, u.y, acc.x));
    acc.y = fmaf(a.x, u.y, fmaf(-a.y, u.x, acc.y));
    acc.z = fmaf(a.x, u.z, fmaf(a.y, u.w, acc.z));
    acc.w = fmaf(a.x, u.w, fmaf(-a.y, u.z, acc.w));
  }
  P[static_cast<size_t>(c) * Npad + m] = acc;
}

__global__ void k_rotate(const float2 *__restrict__ d, int K, float cphi, float sphi,
                         float2 *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) {
    const float2 v = d[k];
    // d e^{-i phi}
    out[k] = make_float2(v.x * cphi + v.y * sphi, v.y * cphi - v.x * sphi);
  }
}

__global__ void k_scale(const float2 *__restrict__ x, float scale, int n, float2 *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(x[i].x * scale, x[i].y * scale);
}

// Number of samples of a pulse with a non-finite component (input validation):
// one workgroup, integer sum.
__global__ __launch_bounds__(256) void k_count_nonfinite(const float2 *__restrict__ d, int K,
                                                         unsigned *__restrict__ count) {
  unsigned n = 0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const float2 v = d[k];
    n += (isfinite(v.x) && isfinite(v.y)) ? 0u : 1u;
  }
  __shared__ unsigned red[256];
  red[threadIdx.x] = n;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = red[0];
}

}  // namespace

hipError_t launch_count_nonfinite(const float2 *d, int K, unsigned *count, hipStream_t st) {
  hipLaunchKernelGGL(k_count_nonfinite, dim3(1), dim3(256), 0, st, d, K, count);
  return hipGetLastError();
}

hipError_t launch_count_large(const float2 *c, int M, float thr, unsigned *count, hipStream_t st) {
  int blocks = (M + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_count_large, dim3(blocks), dim3(256), 0, st, c, M, thr, count);
  return hipGetLastError();
}

hipError_t launch_scale(const float2 *x, float scale, int n, float2 *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, st, x, scale, n, out);
  return hipGetLastError();
}

hipError_t launch_step_tiles(const StepArgs &a, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (a.chunk != 2) return hipErrorInvalidValue;
  auto kern = a.h_cached ? (a.slot_nt ? k_step_tiles<2, true, true> : k_step_tiles<2, true, false>)
                         : (a.slot_nt ? k_step_tiles<2, false, true> : k_step_tiles<2, false, false>);
  if (t0)
    hipExtLaunchKernelGGL(kern, dim3(a.nitems), dim3(256), 0, st, t0, t1, 0, a);
  else
    hipLaunchKernelGGL(kern, dim3(a.nitems), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_steps_resident(const ResidentArgs &a, int nwg, hipStream_t st) {
  if (nwg < 1 || a.iters < 1 || a.iters > kResMaxSteps) return hipErrorInvalidValue;
  ResidentArgs args = a;
  void *params[] = {&args};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_steps_resident), dim3(nwg),
                                    dim3(512), params, 0, st);
}

int resident_grid(int device, int n_cu) {
  int coop = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
      !coop)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(k_steps_resident), 512, 0) != hipSuccess ||
      per_cu < 1)
    return 0;
  return n_cu;
}

hipError_t launch_step_update(const StepArgs &a, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (a.P) {
    if (a.nchunks < 1) return hipErrorInvalidValue;
    if (t0)
      hipExtLaunchKernelGGL(k_step_update<true>, dim3(a.nb * kUpdSplit), dim3(256), 0, st, t0, t1, 0, a);
    else
      hipLaunchKernelGGL(k_step_update<true>, dim3(a.nb * kUpdSplit), dim3(256), 0, st, a);
  } else if (t0) {
    hipExtLaunchKernelGGL(k_step_update<false>, dim3(a.nb * kUpdSplit), dim3(256), 0, st, t0, t1, 0, a);
  } else {
    hipLaunchKernelGGL(k_step_update<false>, dim3(a.nb * kUpdSplit), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_store_forward(const float2 *G, const float2 *D, int rows, int Npad, int M,
                                const float2 *z, const float2 *w, float4 *U, hipStream_t st,
                                hipEvent_t t0, hipEvent_t t1) {
  if (rows <= 0) return hipSuccess;
  const dim3 grid((rows + 3) / 4);
  if (t0)
    hipExtLaunchKernelGGL(k_store_forward, grid, dim3(256), 0, st, t0, t1, 0, G, D, rows, Npad, M, z,
                          w, U);
  else
    hipLaunchKernelGGL(k_store_forward, grid, dim3(256), 0, st, G, D, rows, Npad, M, z, w, U);
  return hipGetLastError();
}

hipError_t launch_store_adjoint(const float2 *G, int rows, int Npad, const float4 *U, float4 *P,
                                hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (rows <= 0) return hipSuccess;
  const dim3 grid((Npad + 255) / 256, (rows + kStoreRows - 1) / kStoreRows);
  if (t0)
    hipExtLaunchKernelGGL(k_store_adjoint, grid, dim3(256), 0, st, t0, t1, 0, G, rows, Npad, U, P);
  else
    hipLaunchKernelGGL(k_store_adjoint, grid, dim3(256), 0, st, G, rows, Npad, U, P);
  return hipGetLastError();
}

hipError_t launch_rotate(const float2 *d, int K, double cos_c, double sin_c, float2 *out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_rotate, dim3((K + 255) / 256), dim3(256), 0, st, d, K,
                     static_cast<float>(cos_c), static_cast<float>(sin_c), out);
  return hipGetLastError();
}

hipError_t launch_scalars(const ScalarArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_scalars, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill(void *p, size_t n_u32, unsigned value, hipStream_t st) {
  if (n_u32 == 0) return hipSuccess;
  size_t blocks = (n_u32 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     static_cast<unsigned *>(p), n_u32, value);
  return hipGetLastError();
}

hipError_t launch_init_power(float2 *w, double *slot0, double *slot1, int N, int Npad, int nparts,
                             hipStream_t st) {
  const int n = Npad > 2 * nparts ? Npad : 2 * nparts;
  hipLaunchKernelGGL(k_init_power, dim3((n + 255) / 256), dim3(256), 0, st, w, slot0, slot1, N,
                     Npad, nparts);
  return hipGetLastError();
}

}  // namespace ofista
