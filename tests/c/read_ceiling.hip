// Read ceiling: what a plain streaming read of B bytes attains on this GPU,
// for comparison with the FISTA tile pass, which reads the packed upper
// triangle of H (4M(M+1) bytes) once per step.
//
//     read_ceiling [MBYTES ...]
//
//     read_ceiling --tiles M [M ...]
//
// With no arguments the sizes are those of H at M = 4096, 7808 and 16384
// coefficients (67.1, 243.9 and 1073.8 MB).  For each size and launch shape
// (workgroups x threads, cached or nontemporal loads) the kernel sums the
// buffer as 16-byte vectors, grid-stride with four loads in flight per
// thread, and writes one partial per workgroup; launches run back to back on
// one stream, each bracketed by events, and the median and mean per launch
// are printed with the byte rate.  The buffer is zero-filled first and the
// first launches are untimed, so a buffer that fits the last-level cache is
// served from there, as H is between FISTA steps.
//
// --tiles reads the same bytes with the tile pass's access pattern and
// nothing else: the packed upper triangle of nb = ceil(M/64) tile rows as
// 64 x 64 tiles of 8-byte elements, one 256-thread workgroup per work item
// (tile row I, runs of two tiles from J = I; the odd last tile of a row
// alone, dispatched after the full runs), wave w loading rows 16w..16w+15 of
// each tile with lane l on column l, every load issued before any is used;
// cached and nontemporal loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int T, bool NT>
__global__ __launch_bounds__(T) void k_read(const f32x4 *__restrict__ p, size_t n16,
                                            float *__restrict__ out) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const size_t stride = static_cast<size_t>(gridDim.x) * T;
  size_t i = static_cast<size_t>(blockIdx.x) * T + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    f32x4 a, b, c, d;
    if constexpr (NT) {
      a = __builtin_nontemporal_load(p + i);
      b = __builtin_nontemporal_load(p + i + stride);
      c = __builtin_nontemporal_load(p + i + 2 * stride);
      d = __builtin_nontemporal_load(p + i + 3 * stride);
    } else {
      a = p[i];
      b = p[i + stride];
      c = p[i + 2 * stride];
      d = p[i + 3 * stride];
    }
    acc += (a + b) + (c + d);
  }
  for (; i < n16; i += stride) acc += p[i];
  __shared__ float red[T];
  red[threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
  __syncthreads();
  for (int o = T / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

#define CHECK(x)                                                                 \
  do {                                                                           \
    const hipError_t err_ = (x);                                                 \
    if (err_ != hipSuccess) {                                                    \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(err_), \
                   __LINE__);                                                    \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

// Tile-pattern read: item i covers tiles t0 .. t0 + n - 1 (n = 1 or 2) of the
// packed tile array (4096 eight-byte elements per tile).
struct TileItem {
  int t0, n;
};
template <bool NT>
__global__ __launch_bounds__(256) void k_read_tiles(const float *__restrict__ H,
                                                    const TileItem *__restrict__ items,
                                                    float *__restrict__ out) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const TileItem it = items[blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  f32x2 h[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const size_t t = static_cast<size_t>(it.t0 + (j < it.n ? j : it.n - 1));
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const f32x2 *ph = reinterpret_cast<const f32x2 *>(H) + t * 4096 + (wave * 16 + q) * 64 + lane;
      if constexpr (NT)
        h[j][q] = __builtin_nontemporal_load(ph);
      else
        h[j][q] = *ph;
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j)
    if (j < it.n)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc += h[j][q].x + h[j][q].y;
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

constexpr int kMaxGrid = 8192;

template <int T, bool NT>
void time_read(const f32x4 *p, size_t bytes, int grid, float *out, int reps) {
  const size_t n16 = bytes / 16;
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto &e : ev) CHECK(hipEventCreate(&e));
  for (int w = 0; w < 5; ++w) hipLaunchKernelGGL((k_read<T, NT>), dim3(grid), dim3(T), 0, 0, p, n16, out);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(ev[2 * r], 0));
    hipLaunchKernelGGL((k_read<T, NT>), dim3(grid), dim3(T), 0, 0, p, n16, out);
    CHECK(hipEventRecord(ev[2 * r + 1], 0));
  }
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  std::vector<float> ms(reps);
  double total = 0.0;
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]));
    total += ms[r];
  }
  std::sort(ms.begin(), ms.end());
  const double med_us = ms[reps / 2] * 1e3, mean_us = total / reps * 1e3;
  std::printf("%10.1f MB  %4d threads  %s  %5d workgroups : median %9.2f us (%5.0f GB/s), "
              "mean %9.2f us (%5.0f GB/s)\n",
              bytes / 1e6, T, NT ? "nontemporal" : "cached     ", grid, med_us,
              bytes / med_us / 1e3, mean_us, bytes / mean_us / 1e3);
  for (auto &e : ev) CHECK(hipEventDestroy(e));
}

template <bool NT>
void time_tiles(const float *H, int M, const TileItem *items, int nitems, size_t bytes, float *out,
                int reps) {
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto &e : ev) CHECK(hipEventCreate(&e));
  for (int w = 0; w < 5; ++w) hipLaunchKernelGGL(k_read_tiles<NT>, dim3(nitems), dim3(256), 0, 0, H, items, out);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(ev[2 * r], 0));
    hipLaunchKernelGGL(k_read_tiles<NT>, dim3(nitems), dim3(256), 0, 0, H, items, out);
    CHECK(hipEventRecord(ev[2 * r + 1], 0));
  }
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  std::vector<float> ms(reps);
  double total = 0.0;
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]));
    total += ms[r];
  }
  std::sort(ms.begin(), ms.end());
  const double med_us = ms[reps / 2] * 1e3, mean_us = total / reps * 1e3;
  std::printf("tiles M = %5d  %10.1f MB  %s  %5d work items : median %9.2f us (%5.0f GB/s), "
              "mean %9.2f us (%5.0f GB/s)\n",
              M, bytes / 1e6, NT ? "nontemporal" : "cached     ", nitems, med_us,
              bytes / med_us / 1e3, mean_us, bytes / mean_us / 1e3);
  for (auto &e : ev) CHECK(hipEventDestroy(e));
}

int tiles_main(int argc, char **argv) {
  std::vector<int> ms;
  for (int a = 2; a < argc; ++a) {
    const int m = std::atoi(argv[a]);
    if (m < 64 || m > 32768) {
      std::fprintf(stderr, "usage: read_ceiling --tiles M [M ...] (each in [64, 32768])\n");
      return 2;
    }
    ms.push_back(m);
  }
  if (ms.empty()) {
    std::fprintf(stderr, "usage: read_ceiling --tiles M [M ...] (each in [64, 32768])\n");
    return 2;
  }
  for (const int m : ms) {
    const int nb = (m + 63) / 64;
    const size_t ntiles = static_cast<size_t>(nb) * (nb + 1) / 2;
    // work items: runs of two from the diagonal; the odd last tiles last
    std::vector<TileItem> full, tail;
    size_t t = 0;
    for (int I = 0; I < nb; ++I) {
      for (int J = I; J < nb; J += 2) {
        const int n = J + 1 < nb ? 2 : 1;
        (n == 2 ? full : tail).push_back({static_cast<int>(t), n});
        t += n;
      }
    }
    full.insert(full.end(), tail.begin(), tail.end());
    if (t != ntiles || full.size() > (size_t{1} << 24)) {
      std::fprintf(stderr, "tile plan mismatch\n");
      return 1;
    }
    const size_t bytes = ntiles * 4096 * 8;
    float *H = nullptr, *out = nullptr;
    TileItem *items = nullptr;
    CHECK(hipMalloc(&H, bytes));
    CHECK(hipMalloc(&out, full.size() * sizeof(float)));
    CHECK(hipMalloc(&items, full.size() * sizeof(TileItem)));
    CHECK(hipMemset(H, 0, bytes));
    CHECK(hipMemcpy(items, full.data(), full.size() * sizeof(TileItem), hipMemcpyHostToDevice));
    const int reps = bytes > (size_t{512} << 20) ? 40 : 200;
    time_tiles<false>(H, m, items, static_cast<int>(full.size()), bytes, out, reps);
    time_tiles<true>(H, m, items, static_cast<int>(full.size()), bytes, out, reps);
    CHECK(hipFree(H));
    CHECK(hipFree(out));
    CHECK(hipFree(items));
  }
  std::printf("done\n");
  return 0;
}

int main(int argc, char **argv) {
  if (argc > 1 && std::string(argv[1]) == "--tiles") return tiles_main(argc, argv);
  std::vector<size_t> sizes;
  for (int a = 1; a < argc; ++a) {
    const double mb = std::atof(argv[a]);
    if (!(mb >= 0.001) || mb > 65536.0) {
      std::fprintf(stderr, "usage: read_ceiling [MBYTES ...] (each in [0.001, 65536])\n");
      return 2;
    }
    sizes.push_back(static_cast<size_t>(mb * 1e6) / 16 * 16);
  }
  if (sizes.empty()) {
    for (const size_t m : {size_t{4096}, size_t{7808}, size_t{16384}}) sizes.push_back(4 * m * (m + 1));
  }
  const size_t maxb = *std::max_element(sizes.begin(), sizes.end());
  f32x4 *p = nullptr;
  float *out = nullptr;
  CHECK(hipMalloc(&p, maxb));
  CHECK(hipMalloc(&out, kMaxGrid * sizeof(float)));
  CHECK(hipMemset(p, 0, maxb));
  CHECK(hipDeviceSynchronize());
  for (const size_t b : sizes) {
    const int reps = b > (size_t{512} << 20) ? 40 : 200;
    for (const int g : {1024, 2048, 4096, kMaxGrid}) {
      time_read<256, false>(p, b, g, out, reps);
      time_read<256, true>(p, b, g, out, reps);
    }
    for (const int g : {1024, 2048}) time_read<512, false>(p, b, g, out, reps);
  }
  CHECK(hipFree(p));
  CHECK(hipFree(out));
  std::printf("done\n");
  return 0;
}
