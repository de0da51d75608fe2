// Exercises the pure-host calls of the ABI (configuration checks, edgelet
// atom enumeration, workspace layout, state-record size) on valid, invalid
// and pseudo-random configurations.  Built together with the library's
// host_plan.cpp under AddressSanitizer and UBSan by tests/test_host_asan.py;
// any out-of-bounds access or undefined behaviour aborts the run.  Exit code
// 0 and "ok" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ofista.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

struct Tables {
  std::vector<double> pos;
  std::vector<int32_t> lens;
  std::vector<double> rots;
};

ofista_config base(Tables &t, int n, int K, int npos) {
  ofista_config c;
  std::memset(&c, 0, sizeof c);
  c.n_x = c.n_y = n;
  c.x0 = c.y0 = -0.5 * n;
  c.dx = c.dy = 1.0;
  t.pos.assign(3 * static_cast<size_t>(npos), 0.0);
  for (int s = 0; s < npos; ++s) {
    t.pos[3 * s] = 1e4 * std::cos(0.001 * s);
    t.pos[3 * s + 1] = 1e4 * std::sin(0.001 * s);
    t.pos[3 * s + 2] = 1e3;
  }
  c.n_pos = npos;
  c.pos_xyz = t.pos.data();
  c.n_freq = K;
  c.freq0_hz = 9.8e9;
  c.dfreq_hz = 1e6;
  c.lambda = 0.05;
  c.lambda_relative = 1;
  return c;
}

void edgelet(ofista_config &c, Tables &t, std::vector<int32_t> lens, std::vector<double> rots) {
  t.lens = lens;
  t.rots = rots;
  c.dict = OFISTA_DICT_EDGELET;
  c.n_edge_lengths = static_cast<int32_t>(t.lens.size());
  c.edge_lengths = t.lens.data();
  c.n_edge_rotations = static_cast<int32_t>(t.rots.size());
  c.edge_rotations_deg = t.rots.data();
}

// one consistent set of answers for a config the library accepts
void consistent(const ofista_config &c, const char *what) {
  const ofista_status st = ofista_check_config(&c);
  const size_t ws = ofista_workspace_bytes(&c);
  const int64_t M = ofista_coef_count(&c);
  const size_t sb = ofista_state_bytes(&c);
  if (st == OFISTA_OK) {
    expect(ws > 0 && M >= 1, what);
    expect(c.storage == OFISTA_STORE_PULSES ? sb == 0 : (sb > 0 && sb <= ws), what);
  } else {
    expect(ws == 0 && M == -1 && sb == 0, what);
  }
}

}  // namespace

int main() {
  Tables t;
  expect(ofista_tile() == 64, "tile edge");
  expect(ofista_check_config(nullptr) == OFISTA_E_ARG, "null config");
  expect(ofista_workspace_bytes(nullptr) == 0, "null config bytes");

  // valid shapes of every dictionary, precision and storage
  for (int n : {1, 7, 16, 30, 64}) {
    ofista_config c = base(t, n, 32, 5);
    expect(ofista_check_config(&c) == OFISTA_OK, "identity");
    expect(ofista_coef_count(&c) == static_cast<int64_t>(n) * n, "identity M");
    consistent(c, "identity");
    c.precision = OFISTA_PREC_SPLIT_BF16;
    for (int lay : {OFISTA_GRAM_AUTO, OFISTA_GRAM_TILE, OFISTA_GRAM_BLOCK}) {
      c.gram_layout = lay;
      expect(ofista_check_config(&c) == OFISTA_OK, "split-BF16 layouts");
      consistent(c, "split-BF16");
    }
    c.gram_layout = 0;
    c.precision = OFISTA_PREC_FP32;
    c.storage = OFISTA_STORE_PULSES;
    c.max_pulses = 3;
    consistent(c, "pulses storage");
    c.storage = OFISTA_STORE_GRAM;
    c.record_every = 2;
    c.max_pulses = 5;
    c.max_iters = 4;
    consistent(c, "recording");
  }
  {
    ofista_config c = base(t, 32, 64, 3);
    c.dict = OFISTA_DICT_HAAR2D;
    c.haar_levels = 3;
    expect(ofista_check_config(&c) == OFISTA_OK, "haar");
    consistent(c, "haar");
    c.haar_levels = 6;
    expect(ofista_check_config(&c) == OFISTA_E_ARG, "haar levels");
  }
  // edgelets: closed-form counts n (n - l + 1) for each axis-aligned rotation
  for (int n : {2, 5, 16, 33}) {
    for (int l = 1; l <= n - 1; l += (n > 8 ? 5 : 1)) {
      ofista_config c = base(t, n, 16, 2);
      edgelet(c, t, {l}, {0.0, 90.0});
      expect(ofista_coef_count(&c) == 2LL * n * (n - l + 1), "edgelet axis count");
      consistent(c, "edgelet");
    }
  }
  {
    ofista_config c = base(t, 24, 16, 2);
    edgelet(c, t, {2, 3, 5}, {30.0, 45.0, 100.0, 135.0, -720.0});
    consistent(c, "oblique edgelets");
    edgelet(c, t, {24}, {0.0});
    expect(ofista_check_config(&c) == OFISTA_E_ARG, "edgelet length out of range");
    edgelet(c, t, {4}, {NAN});
    expect(ofista_check_config(&c) == OFISTA_E_ARG, "edgelet NaN rotation");
    c.edge_lengths = nullptr;
    expect(ofista_check_config(&c) == OFISTA_E_ARG, "edgelet NULL lengths");
  }
  // invalid fields
  {
    ofista_config c = base(t, 16, 32, 4);
    ofista_config b = c;
    b.n_freq = 0;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "K = 0");
    b = c;
    b.n_freq = 2048;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "K too large");
    b = c;
    b.pos_xyz = nullptr;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "NULL positions");
    b = c;
    t.pos[4] = NAN;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "NaN position");
    t.pos[4] = 0.0;
    b = c;
    b.gram_layout = 7;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "layout value");
    b = c;
    b.gram_layout = OFISTA_GRAM_BLOCK;
    expect(ofista_check_config(&b) == OFISTA_E_UNSUPPORTED, "layout with FP32");
    b = c;
    b.precision = OFISTA_PREC_SPLIT_BF16;
    b.n_freq = 50;
    expect(ofista_check_config(&b) == OFISTA_E_UNSUPPORTED, "split-BF16 ragged K");
    b = c;
    b.n_x = 1 << 10;
    b.n_y = 1 << 10;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "N too large");
    b = c;
    b.lambda = -1.0;
    expect(ofista_check_config(&b) == OFISTA_E_ARG, "negative lambda");
  }
  // pseudo-random configurations (fixed LCG): no crash, consistent answers
  uint64_t x = 2603;
  auto next = [&](int mod) {
    x = x * 6364136223846793005ULL + 1442695040888963407ULL;
    return static_cast<int>((x >> 33) % static_cast<uint64_t>(mod));
  };
  for (int it = 0; it < 400; ++it) {
    const int n = 1 + next(40);
    ofista_config c = base(t, n, 1 + next(1100), 1 + next(6));
    c.n_y = 1 + next(40);
    c.dict = next(3);
    c.haar_levels = next(4);
    c.precision = next(3) == 0 ? OFISTA_PREC_SPLIT_BF16 : OFISTA_PREC_FP32;
    c.gram_layout = next(4) == 0 ? next(4) : 0;
    c.storage = next(4) == 0 ? OFISTA_STORE_PULSES : OFISTA_STORE_GRAM;
    c.max_pulses = next(6);
    c.max_iters = next(4);
    c.record_every = next(5) == 0 ? next(3) : 0;
    c.backprojection = next(2);
    if (c.dict == OFISTA_DICT_EDGELET) {
      c.n_y = c.n_x;
      std::vector<int32_t> lens;
      std::vector<double> rots;
      for (int k = 0, m = 1 + next(3); k < m; ++k) lens.push_back(next(n + 2));
      for (int k = 0, m = 1 + next(3); k < m; ++k) rots.push_back(next(360) - 180.0);
      edgelet(c, t, lens, rots);
    }
    consistent(c, "random");
  }
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
