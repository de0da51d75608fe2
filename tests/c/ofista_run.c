/*
 * ofista_run -- drives libofista through its C ABI from plain C (no Python,
 * no PyTorch): device memory and the stream come from the HIP runtime API.
 *
 *   ofista_run FILE OUT     run the problem described in FILE (written by the
 *                           test suite), write the final image (N complex64)
 *                           to OUT
 *   ofista_run --haar64 P   the 64 x 64 Haar workload shape (K = 256, 128
 *                           positions over 20 degrees at 10 km, m = 20) with P
 *                           pushed pulses of seeded pseudo-random data: a
 *                           fixed, self-contained launch sequence for counter
 *                           collection
 *   ofista_run --xlarge P   the 256 x 256 identity workload shape (K = 1024,
 *                           512 positions over 40 degrees, m = 10, split-BF16
 *                           Gram update) with P pushed pulses of seeded data
 *   ofista_run --copy MIB   one device-to-device copy of MIB MiB (the known
 *                           byte count that scales the memory counters)
 *
 * FILE layout (little-endian): int32 n_x, n_y; double x0, y0, dx, dy;
 * int32 n_pos, n_freq; double freq0, dfreq; int32 dict, haar_levels;
 * double lambda; int32 lambda_relative, iters, n_push; double pos[n_pos*3];
 * int32 order[n_push]; float pulses[n_push*n_freq*2].
 *
 * Exit status 0 on success, 1 on usage/IO errors, 2 on library or HIP errors
 * (the message goes to stderr).
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ofista.h"

#define HIP_OK(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                \
      exit(2);                                                                  \
    }                                                                           \
  } while (0)

static void lib_ok(struct ofista_ctx *ctx, ofista_status st, const char *what) {
  if (st != OFISTA_OK) {
    fprintf(stderr, "%s: %s\n", what, ofista_error_string(ctx, st));
    exit(2);
  }
}

static int read_all(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

typedef struct problem {
  ofista_config cfg;
  int32_t iters, n_push;
  double *pos;
  int32_t *order;
  float *pulses; /* n_push x n_freq complex64 */
} problem;

static int load(const char *path, problem *pb) {
  FILE *f = fopen(path, "rb");
  if (!f) return 0;
  ofista_config *c = &pb->cfg;
  memset(pb, 0, sizeof *pb);
  int ok = read_all(f, &c->n_x, 4) && read_all(f, &c->n_y, 4) && read_all(f, &c->x0, 8) &&
           read_all(f, &c->y0, 8) && read_all(f, &c->dx, 8) && read_all(f, &c->dy, 8) &&
           read_all(f, &c->n_pos, 4) && read_all(f, &c->n_freq, 4) && read_all(f, &c->freq0_hz, 8) &&
           read_all(f, &c->dfreq_hz, 8) && read_all(f, &c->dict, 4) && read_all(f, &c->haar_levels, 4) &&
           read_all(f, &c->lambda, 8) && read_all(f, &c->lambda_relative, 4) &&
           read_all(f, &pb->iters, 4) && read_all(f, &pb->n_push, 4);
  if (ok && (c->n_pos < 1 || c->n_freq < 1 || pb->n_push < 0)) ok = 0;
  if (ok) {
    pb->pos = malloc(sizeof(double) * 3 * (size_t)c->n_pos);
    pb->order = malloc(sizeof(int32_t) * (size_t)(pb->n_push + 1));
    pb->pulses = malloc(sizeof(float) * 2 * (size_t)c->n_freq * (size_t)(pb->n_push + 1));
    ok = pb->pos && pb->order && pb->pulses &&
         read_all(f, pb->pos, sizeof(double) * 3 * (size_t)c->n_pos) &&
         read_all(f, pb->order, sizeof(int32_t) * (size_t)pb->n_push) &&
         read_all(f, pb->pulses, sizeof(float) * 2 * (size_t)c->n_freq * (size_t)pb->n_push);
  }
  fclose(f);
  c->pos_xyz = pb->pos;
  return ok;
}

/* A square identity or Haar workload shape on the 10 km / 1 km circle, with
   pulse data from a 64-bit LCG. */
static void synthetic(problem *pb, int32_t n_push, int n, int P, int K, double patch,
                      double arc_deg, double f_lo, double f_hi, int dict, int levels,
                      int precision, int iters) {
  ofista_config *c = &pb->cfg;
  memset(pb, 0, sizeof *pb);
  const double dxy = patch / n, pi = 3.14159265358979323846;
  c->n_x = c->n_y = n;
  c->x0 = c->y0 = -patch / 2 + dxy / 2;
  c->dx = c->dy = dxy;
  c->n_pos = P;
  pb->pos = malloc(sizeof(double) * 3 * P);
  for (int s = 0; s < P; ++s) {
    const double th = s * (arc_deg * pi / 180.0) / (P - 1);
    pb->pos[3 * s] = 10000.0 * cos(th);
    pb->pos[3 * s + 1] = 10000.0 * sin(th);
    pb->pos[3 * s + 2] = 1000.0;
  }
  c->pos_xyz = pb->pos;
  c->n_freq = K;
  c->freq0_hz = f_lo;
  c->dfreq_hz = (f_hi - f_lo) / (K - 1);
  c->dict = dict;
  c->haar_levels = levels;
  c->precision = precision;
  c->lambda = 0.05;
  c->lambda_relative = 1;
  pb->iters = iters;
  pb->n_push = n_push;
  pb->order = malloc(sizeof(int32_t) * (size_t)(n_push + 1));
  pb->pulses = malloc(sizeof(float) * 2 * (size_t)K * (size_t)(n_push + 1));
  uint64_t x = 2603;
  for (int32_t p = 0; p < n_push; ++p) {
    pb->order[p] = p % P;
    for (int k = 0; k < 2 * K; ++k) {
      x = x * 6364136223846793005ULL + 1442695040888963407ULL;
      pb->pulses[(size_t)p * 2 * K + k] = (float)((double)(x >> 11) / 9007199254740992.0 - 0.5);
    }
  }
}

static int copy_once(int mib) {
  const size_t bytes = (size_t)mib << 20;
  void *a = NULL, *b = NULL;
  HIP_OK(hipMalloc(&a, bytes));
  HIP_OK(hipMalloc(&b, bytes));
  HIP_OK(hipMemset(a, 1, bytes));
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(b, a, bytes, hipMemcpyDeviceToDevice));
  HIP_OK(hipDeviceSynchronize());
  printf("copied %d MiB\n", mib);
  HIP_OK(hipFree(a));
  HIP_OK(hipFree(b));
  return 0;
}

int main(int argc, char **argv) {
  problem pb;
  const char *out = NULL;
  if (argc == 3 && strcmp(argv[1], "--copy") == 0) {
    const int mib = atoi(argv[2]);
    return mib >= 1 && mib <= 4096 ? copy_once(mib) : 1;
  }
  if (argc == 3 && strcmp(argv[1], "--haar64") == 0) {
    const int n = atoi(argv[2]);
    if (n < 1) return 1;
    synthetic(&pb, n, 64, 128, 256, 60.0, 20.0, 9.8e9, 10.2e9, OFISTA_DICT_HAAR2D, 3,
              OFISTA_PREC_FP32, 20);
  } else if (argc == 3 && strcmp(argv[1], "--xlarge") == 0) {
    const int n = atoi(argv[2]);
    if (n < 1) return 1;
    synthetic(&pb, n, 256, 512, 1024, 250.0, 40.0, 9.7e9, 10.3e9, OFISTA_DICT_IDENTITY, 0,
              OFISTA_PREC_SPLIT_BF16, 10);
  } else if (argc == 3) {
    if (!load(argv[1], &pb)) {
      fprintf(stderr, "cannot read %s\n", argv[1]);
      return 1;
    }
    out = argv[2];
  } else {
    fprintf(stderr, "usage: ofista_run FILE OUT | ofista_run --haar64 PULSES | ofista_run --xlarge PULSES | ofista_run --copy MIB\n");
    return 1;
  }
  ofista_config *c = &pb.cfg;
  const size_t ws = ofista_workspace_bytes(c);
  const int64_t M = ofista_coef_count(c);
  if (ws == 0 || M < 1) {
    fprintf(stderr, "invalid configuration: %s\n", ofista_error_string(NULL, ofista_check_config(c)));
    return 2;
  }
  const size_t N = (size_t)c->n_x * (size_t)c->n_y, K = (size_t)c->n_freq;
  hipStream_t st;
  void *d_ws = NULL, *d_pulses = NULL, *d_img = NULL;
  HIP_OK(hipStreamCreate(&st));
  HIP_OK(hipMalloc(&d_ws, ws));
  HIP_OK(hipMalloc(&d_pulses, 8 * K * (size_t)(pb.n_push > 0 ? pb.n_push : 1)));
  HIP_OK(hipMalloc(&d_img, 8 * N));
  if (pb.n_push > 0)
    HIP_OK(hipMemcpy(d_pulses, pb.pulses, 8 * K * (size_t)pb.n_push, hipMemcpyHostToDevice));
  struct ofista_ctx *ctx = NULL;
  lib_ok(ctx, ofista_create(c, d_ws, ws, st, &ctx), "ofista_create");
  for (int32_t p = 0; p < pb.n_push; ++p) {
    lib_ok(ctx, ofista_push_pulse(ctx, (const char *)d_pulses + 8 * K * (size_t)p, pb.order[p], 0.0),
           "ofista_push_pulse");
    lib_ok(ctx, ofista_reconstruct(ctx, pb.iters, NULL), "ofista_reconstruct");
  }
  ofista_stats stats;
  if (pb.n_push > 0) lib_ok(ctx, ofista_image(ctx, d_img), "ofista_image");
  lib_ok(ctx, ofista_state(ctx, &stats), "ofista_state");
  printf("pulses %lld steps %lld L %.9g lambda %.9g\n", (long long)stats.n_pulses,
         (long long)stats.n_iters, stats.L, stats.lambda);
  int rc = 0;
  if (out) {
    float *img = malloc(8 * N);
    HIP_OK(hipMemcpy(img, d_img, 8 * N, hipMemcpyDeviceToHost));
    FILE *f = fopen(out, "wb");
    if (!f || fwrite(img, 8, N, f) != N) rc = 1;
    if (f) fclose(f);
    free(img);
  }
  ofista_destroy(ctx);
  HIP_OK(hipFree(d_img));
  HIP_OK(hipFree(d_pulses));
  HIP_OK(hipFree(d_ws));
  HIP_OK(hipStreamDestroy(st));
  free(pb.pos);
  free(pb.order);
  free(pb.pulses);
  return rc;
}
