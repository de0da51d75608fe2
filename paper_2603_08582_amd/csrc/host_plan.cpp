// Host-side plan of libofista: configuration checks, edgelet atom tables,
// workspace layout and the pure-host calls of the ABI (no GPU needed).
#include "host_plan.h"

#include <algorithm>
#include <cmath>

namespace ofista {

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t state_record_bytes(const Layout &L) {
  return align_up(16 * sizeof(double)) + align_up(sizeof(DevScalars)) +
         2 * align_up(2 * L.nparts * sizeof(double)) +
         3 * align_up(static_cast<size_t>(L.Npad) * kBytesC64) +
         align_up(L.ntiles * kTile * kTile * kBytesC64) +
         (L.has_bp ? align_up(static_cast<size_t>(L.npix) * kBytesC64) : 0);
}

size_t count_items(int nb, int chunk) {
  size_t n = 0;
  for (int I = 0; I < nb; ++I) n += static_cast<size_t>((nb - I + chunk - 1) / chunk);
  return n;
}

// Edgelet atoms of the dictionary (rule in include/ofista.h): pixel lists
// in atom order.  Returns the atom count, or -1 when a length is out of range.
// Floating-point contraction is off so that every rounding happens in the
// order written (x0 + u*c, then + 0.5, then - 1e-9).
long long edgelet_atoms(const ofista_config *c, std::vector<int> *ptr, std::vector<int> *pix) {
#pragma clang fp contract(off)
  const int n = c->n_x;
  const double kDeg = 3.14159265358979323846 / 180.0;
  long long M = 0;
  std::vector<int> one;
  if (ptr) ptr->assign(1, 0);
  if (pix) pix->clear();
  for (int r = 0; r < c->n_edge_rotations; ++r) {
    const double psi = c->edge_rotations_deg[r] * kDeg;
    const double cs = std::cos(psi), sn = std::sin(psi);
    for (int li = 0; li < c->n_edge_lengths; ++li) {
      const int len = c->edge_lengths[li];
      if (len < 1 || len > n - 1) return -1;
      for (int y0 = 0; y0 < n; ++y0)
        for (int x0 = 0; x0 < n; ++x0) {
          one.clear();
          bool inside = true;
          for (int t = 0; t < len && inside; ++t) {
            const double u = t - (len - 1) / 2.0;
            const double vx = x0 + u * cs;
            const double vy = y0 + u * sn;
            const long long ix = static_cast<long long>(std::floor(vx + 0.5 - 1e-9));
            const long long iy = static_cast<long long>(std::floor(vy + 0.5 - 1e-9));
            if (ix < 0 || ix >= n || iy < 0 || iy >= n) inside = false;
            else one.push_back(static_cast<int>(iy * n + ix));
          }
          if (!inside) continue;
          std::sort(one.begin(), one.end());
          one.erase(std::unique(one.begin(), one.end()), one.end());
          ++M;
          if (pix) pix->insert(pix->end(), one.begin(), one.end());
          if (ptr) ptr->push_back(static_cast<int>(pix ? pix->size() : 0));
        }
    }
  }
  return M;
}

// Coefficient count and total atom pixels for a checked config.
long long coef_count(const ofista_config *c, size_t *nnz) {
  if (c->dict != OFISTA_DICT_EDGELET) {
    if (nnz) *nnz = 0;
    return static_cast<long long>(c->n_x) * c->n_y;
  }
  std::vector<int> ptr, pix;
  const long long M = edgelet_atoms(c, &ptr, &pix);
  if (nnz) *nnz = pix.size();
  return M;
}

// The split-BF16 Gram switches to 2 x 2 tile blocks (one tile per wave) from
// this many tile rows on: measured faster at N = 16384 and 65536, slower at
// N = 4096.
constexpr int kBfBlockMinNb = 256;

// FP32 Gram remainder split.  With q whole rounds of one tile per CU and a
// remainder r, the r tiles of the last round run nearly alone on their CUs,
// latency-bound: at N = 4096 (2080 tiles = 8 x 256 + 32) they cost 20 us of
// 168.  Splitting r off-diagonal tiles into up to 8 frequency pieces that run
// after the whole tiles shortens that tail (measured: 168 -> 158 us with the
// pieces in a separate launch).  Beyond kSplitMaxRounds rounds the remainder
// costs under 1% and the tiles are left whole; below 2 rounds every tile is
// resident from the start and there is no tail of lone tiles.
constexpr size_t kGramCUs = 256;  // compute units of the MI355X
constexpr size_t kSplitMaxRounds = 64;
constexpr int kSplitParts = kGramSplitMaxParts;

void plan_gram_split(Layout &L) {
  L.gram_grid = L.ntiles_grid;
  const size_t q = L.ntiles / kGramCUs, rem = L.ntiles % kGramCUs;
  const int parts = std::min((L.K + L.gram_kb - 1) / L.gram_kb, kSplitParts);
  if (q < 2 || q >= kSplitMaxRounds || rem == 0 || parts < 2 || rem > L.ntiles - L.nb) return;
  L.gsplit = rem;
  L.gparts = parts;
  const size_t whole = L.ntiles - rem;  // q * kGramCUs, a multiple of 8
  L.gram_grid = 8 * (whole / 8 + (rem * parts + 7) / 8);
}

// Run length of the FISTA work items.  Runs of 2 tiles measured faster than
// runs of 4 or 8 at both N = 4096 and N = 16384 (more workgroups in flight).
int pick_chunk(int) { return kChunk; }

ofista_status check(const ofista_config *c, std::string *why) {
  auto bad = [&](const char *m) {
    if (why) *why = m;
    return OFISTA_E_ARG;
  };
  if (!c) return bad("config is NULL");
  if (c->n_x < 1 || c->n_y < 1) return bad("n_x and n_y must be >= 1");
  const long long N = static_cast<long long>(c->n_x) * c->n_y;
  if (N > (1LL << 18)) return bad("N = n_x*n_y must be <= 262144");
  if (!std::isfinite(c->x0) || !std::isfinite(c->y0) || !std::isfinite(c->dx) ||
      !std::isfinite(c->dy))
    return bad("grid origin and spacing must be finite");
  if (c->n_pos < 1) return bad("n_pos must be >= 1");
  if (!c->pos_xyz) return bad("pos_xyz is NULL");
  if (c->n_freq < 1 || c->n_freq > kMaxFreq) return bad("n_freq must be in [1, 1024]");
  if (!std::isfinite(c->freq0_hz) || !std::isfinite(c->dfreq_hz))
    return bad("frequencies must be finite");
  if (c->dict != OFISTA_DICT_IDENTITY && c->dict != OFISTA_DICT_HAAR2D &&
      c->dict != OFISTA_DICT_EDGELET)
    return bad("unknown dict");
  if (c->dict == OFISTA_DICT_EDGELET) {
    if (c->n_x != c->n_y) return bad("edgelet dictionary needs a square grid");
    if (c->n_x < 2) return bad("edgelet dictionary needs n_x >= 2");
    if (c->n_edge_lengths < 1 || !c->edge_lengths) return bad("edgelet lengths missing");
    if (c->n_edge_rotations < 1 || !c->edge_rotations_deg) return bad("edgelet rotations missing");
    if (static_cast<long long>(c->n_edge_lengths) * c->n_edge_rotations > 4096)
      return bad("too many edgelet lengths x rotations");
    for (int i = 0; i < c->n_edge_lengths; ++i)
      if (c->edge_lengths[i] < 1 || c->edge_lengths[i] > c->n_x - 1)
        return bad("edgelet lengths must be in [1, n_x - 1]");
    for (int i = 0; i < c->n_edge_rotations; ++i)
      if (!std::isfinite(c->edge_rotations_deg[i])) return bad("edgelet rotations must be finite");
    const long long M = edgelet_atoms(c, nullptr, nullptr);
    if (M < 1) return bad("the edgelet dictionary has no atom on this grid");
    if (M > (1LL << 18)) {
      if (why) *why = "edgelet dictionary limited to M <= 262144 atoms";
      return OFISTA_E_UNSUPPORTED;
    }
    // the per-position K x K FP64 matrices of sigma^2 borrow the H region
    // (the stored-pulse region when storing pulses)
    const long long nbm = (M + kTile - 1) / kTile;
    const long long hbytes = c->storage == OFISTA_STORE_PULSES
                                 ? static_cast<long long>(c->max_pulses) * c->n_freq * nbm * kTile * 8
                                 : nbm * (nbm + 1) / 2 * kTile * kTile * 8;
    if (static_cast<long long>(c->n_freq) * c->n_freq * 16 > hbytes) {
      if (why) *why = "edgelet dictionary: K*K*16 bytes exceed the H storage";
      return OFISTA_E_UNSUPPORTED;
    }
  }
  if (c->dict == OFISTA_DICT_HAAR2D) {
    if (c->haar_levels < 1) return bad("haar_levels must be >= 1");
    if (c->n_x != c->n_y) return bad("Haar dictionary needs a square grid");
    if (c->haar_levels > 14 || c->n_x % (1 << c->haar_levels) != 0)
      return bad("n_x must be divisible by 2^haar_levels");
    if (N > 8192) {
      if (why) *why = "Haar dictionary is limited to N <= 8192";
      return OFISTA_E_UNSUPPORTED;
    }
  }
  if (!std::isfinite(c->lambda) || c->lambda < 0) return bad("lambda must be finite and >= 0");
  if (c->precision != OFISTA_PREC_FP32 && c->precision != OFISTA_PREC_SPLIT_BF16)
    return bad("unknown precision");
  if (c->lipschitz != OFISTA_LIP_RUNNING && c->lipschitz != OFISTA_LIP_BOUND)
    return bad("unknown lipschitz rule");
  if (c->momentum < OFISTA_MOMENTUM_FISTA || c->momentum > OFISTA_MOMENTUM_ISTA)
    return bad("unknown momentum mode");
  if (c->record_every < 0) return bad("record_every must be >= 0");
  if (c->gram_layout < OFISTA_GRAM_AUTO || c->gram_layout > OFISTA_GRAM_BLOCK)
    return bad("unknown gram_layout");
  if (c->gram_layout != OFISTA_GRAM_AUTO && c->precision != OFISTA_PREC_SPLIT_BF16) {
    if (why) *why = "gram_layout selects among the split-BF16 Gram kernels only";
    return OFISTA_E_UNSUPPORTED;
  }
  if (c->step_kernel < OFISTA_STEP_AUTO || c->step_kernel > OFISTA_STEP_RESIDENT)
    return bad("unknown step_kernel");
  if (c->step_kernel == OFISTA_STEP_RESIDENT && c->storage == OFISTA_STORE_PULSES) {
    if (why) *why = "the resident step kernel works on the Gram storage only";
    return OFISTA_E_UNSUPPORTED;
  }
  if (c->precision == OFISTA_PREC_SPLIT_BF16 && c->n_freq % 32 != 0) {
    if (why) *why = "split-BF16 Gram update needs n_freq divisible by 32";
    return OFISTA_E_UNSUPPORTED;
  }
  if (c->record_every > 0 && (c->max_pulses < 1 || c->max_iters < 1))
    return bad("recording needs max_pulses >= 1 and max_iters >= 1");
  for (int i = 0; i < 3 * c->n_pos; ++i)
    if (!std::isfinite(c->pos_xyz[i])) return bad("pos_xyz must be finite");
  if (c->storage != OFISTA_STORE_GRAM && c->storage != OFISTA_STORE_PULSES) return bad("unknown storage");
  if (c->storage == OFISTA_STORE_PULSES) {
    if (c->max_pulses < 1) return bad("storing pulses needs max_pulses >= 1");
    if (c->record_every != 0 || c->precision != OFISTA_PREC_FP32) {
      if (why) *why = "storing pulses excludes recording and the split-BF16 Gram";
      return OFISTA_E_UNSUPPORTED;
    }
  }
  return OFISTA_OK;
}

Layout layout(const ofista_config *c) {
  Layout L;
  L.npix = c->n_x * c->n_y;
  L.N = static_cast<int>(coef_count(c, &L.nnz));
  L.nb = (L.N + kTile - 1) / kTile;
  L.Npad = L.nb * kTile;
  L.K = c->n_freq;
  L.npos = c->n_pos;
  L.store = c->storage == OFISTA_STORE_PULSES;
  L.ntiles = L.store ? 0 : static_cast<size_t>(L.nb) * (L.nb + 1) / 2;
  L.ntiles_grid = (L.ntiles + 7) / 8 * 8;
  L.gram_grid = L.ntiles_grid;
  {
    const size_t hbytes = L.ntiles * kTile * kTile * kBytesC64;
    L.gram_kb = hbytes <= kLlcBytes / 2 ? kGramKBSmall : kGramKBLarge;
    L.h_cached = hbytes <= kLlcBytes;
    // partial slots beyond the last-level cache are read back from HBM by the
    // update anyway: written nontemporal they stay out of the tile pass's
    // read stream (xlarge: 3.12 against 3.28 ms per pass); slots that fit are
    // read back from the cache, which nontemporal stores would give up
    // (large: the update lost more than the pass gained)
    const size_t slot_bytes = static_cast<size_t>(L.nb) * L.nb * kTile * kBytesF4;
    L.slot_nt = slot_bytes > kLlcBytes;
  }
  if (!L.store && c->precision == OFISTA_PREC_FP32) plan_gram_split(L);
  L.chunk = pick_chunk(L.nb);
  L.nparts = kUpdSplit * L.nb;
  L.nitems = count_items(L.nb, L.chunk);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t vec = static_cast<size_t>(L.Npad) * kBytesC64;
  L.H = take(L.ntiles * kTile * kTile * kBytesC64);
  L.A = take(static_cast<size_t>(L.K) * L.Npad * kBytesC64);
  L.b = take(vec);
  L.c0 = take(vec);
  L.c1 = take(vec);
  L.z0 = take(vec);
  L.z1 = take(vec);
  L.w0 = take(vec);
  L.w1 = take(vec);
  L.Q = take(L.store ? 0 : static_cast<size_t>(L.nb) * L.nb * kTile * kBytesF4);
  if (L.store) {
    L.store_cap = c->max_pulses;
    const size_t rows = static_cast<size_t>(L.store_cap) * L.K;
    L.store_chunks = static_cast<int>((rows + kStoreRows - 1) / kStoreRows);
    L.Gst = take(rows * L.Npad * kBytesC64);
    L.Dst = take(rows * kBytesC64);
    L.Ust = take(rows * kBytesF4);
    L.Pst = take(static_cast<size_t>(L.store_chunks) * L.Npad * kBytesF4);
  }
  L.slot0 = take(2 * L.nparts * sizeof(double));
  L.slot1 = take(2 * L.nparts * sizeof(double));
  L.scal = take(sizeof(DevScalars));
  L.pos = take(3 * static_cast<size_t>(L.npos) * sizeof(double));
  L.sig2 = take(L.npos * sizeof(double));
  L.gtoep = take(static_cast<size_t>(L.npos) * L.K * kBytesD2);
  L.tile_ij = take(std::max(L.ntiles_grid, L.gram_grid) * kBytesI2);
  L.gP = take(L.gsplit * L.gparts * kTile * kTile * kBytesC64);
  L.gsplit_ij = take(L.gsplit * kBytesI2);
  L.tile_row0 = take(L.nb * sizeof(int));
  L.items = take(L.nitems * sizeof(WorkItem));
  L.echo_tmp = take(L.K * kBytesD2);
  L.counter = take(sizeof(unsigned));
  L.bar = take(8 * kBarStride * sizeof(unsigned));
  L.has_bp = c->backprojection != 0;
  if (L.has_bp) L.bp = take(static_cast<size_t>(L.npix) * kBytesC64);
  if (c->dict == OFISTA_DICT_EDGELET) {
    L.atom_ptr = take((static_cast<size_t>(L.N) + 1) * sizeof(int));
    L.atom_pix = take(L.nnz * sizeof(int));
    L.pix_ptr = take((static_cast<size_t>(L.npix) + 1) * sizeof(int));
    L.pix_atom = take(L.nnz * sizeof(int));
  }
  L.Ahi = L.Alo = 0;
  const bool bf_blocked = c->gram_layout == OFISTA_GRAM_BLOCK ||
                          (c->gram_layout == OFISTA_GRAM_AUTO && L.nb >= kBfBlockMinNb);
  if (c->precision == OFISTA_PREC_SPLIT_BF16 && bf_blocked) {
    const size_t nbB = (L.nb + 1) / 2;
    // the launch grid: the nbB (nbB + 1) / 2 blocks padded to a multiple of
    // 8, one run per XCD
    L.nbf_blocks = (nbB * (nbB + 1) / 2 + 7) / 8 * 8;
    L.bf_blocks = take(L.nbf_blocks * kBytesI2);
  }
  if (c->precision == OFISTA_PREC_SPLIT_BF16) {
    L.Ahi = take(static_cast<size_t>(L.Npad) * L.K * sizeof(unsigned));
    L.Alo = take(static_cast<size_t>(L.Npad) * L.K * sizeof(unsigned));
  }
  L.state_bytes = state_record_bytes(L);
  if (c->record_every > 0) {
    L.rec_every = c->record_every;
    L.rec_pulses = c->max_pulses;
    L.rec_iters = c->max_iters;
    L.n_ckpt = (L.rec_pulses + L.rec_every - 1) / L.rec_every + 1;  // + the live state
    const int R = std::min(L.rec_every, L.rec_pulses);
    L.ckpt = take(static_cast<size_t>(L.n_ckpt) * align_up(L.state_bytes));
    L.pulses_d = take(static_cast<size_t>(L.rec_pulses) * L.K * kBytesC64);
    L.seg_H = take(static_cast<size_t>(R) * L.ntiles * kTile * kTile * kBytesC64);
    L.seg_u = take(static_cast<size_t>(R) * L.rec_iters * vec);
    L.seg_db = take(static_cast<size_t>(R) * vec);
    L.seg_scal = take(static_cast<size_t>(R) * sizeof(DevScalars));
    L.chat_bar = take(vec);
    L.ubar0 = take(vec);
    L.ubar1 = take(vec);
    L.cpart0 = take(vec);
    L.cpart1 = take(vec);
    L.bbar = take(vec);
    L.Bbar = take(vec);
    L.alpha_parts = take(static_cast<size_t>(L.rec_iters) * L.nb * sizeof(double));
    L.lam_dev = take(static_cast<size_t>(L.rec_pulses) * sizeof(double));
    L.phase_dev = take(static_cast<size_t>(L.rec_pulses) * sizeof(double));
  }
  L.total = o;
  return L;
}

const char *status_text(ofista_status st) {
  switch (st) {
    case OFISTA_OK: return "ok";
    case OFISTA_E_ARG: return "invalid argument";
    case OFISTA_E_RANGE: return "pulse index out of range";
    case OFISTA_E_STATE: return "call not valid in the current state";
    case OFISTA_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case OFISTA_E_UNSUPPORTED: return "unsupported configuration";
    case OFISTA_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}


}  // namespace ofista

using namespace ofista;

extern "C" {

int32_t ofista_tile(void) { return kTile; }

ofista_status ofista_check_config(const ofista_config *cfg) { return check(cfg, nullptr); }

int64_t ofista_coef_count(const ofista_config *cfg) {
  if (check(cfg, nullptr) != OFISTA_OK) return -1;
  return coef_count(cfg, nullptr);
}

size_t ofista_workspace_bytes(const ofista_config *cfg) {
  if (check(cfg, nullptr) != OFISTA_OK) return 0;
  return layout(cfg).total;
}

size_t ofista_state_bytes(const ofista_config *cfg) {
  if (check(cfg, nullptr) != OFISTA_OK || cfg->storage == OFISTA_STORE_PULSES) return 0;
  return state_record_bytes(layout(cfg));
}

}  // extern "C"
