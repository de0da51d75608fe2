// Host-side plan of libofista: configuration checks, the edgelet atom
// tables, the workspace layout and the sizes behind the pure-host calls of
// the ABI.  Plain C++ with no HIP dependency, so that it also builds with the
// host compiler alone (the AddressSanitizer check of the CPU tests does).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ofista.h"

namespace ofista {

// Edge of the square tiles of the packed Hermitian storage.  H is kept as
// the nb(nb+1)/2 tiles (I, J), I <= J, of a zero-padded Npad x Npad matrix
// (Npad = nb * kTile), each tile row-major, tiles in row-major upper order.
constexpr int kTile = 64;

// Tiles per FISTA work item (a run of tiles along one tile row): 2 or 4.
constexpr int kChunk = 2;
// Workgroups per tile row in the FISTA update; the power-iteration parts
// (slots) are kept per update workgroup: nparts = kUpdSplit * nb.
constexpr int kUpdSplit = 4;
// Frequencies staged per LDS step of the FP32 Gram update, and whether the
// FISTA tile pass reads H with cached loads, by the size of the packed H
// against the 256 MB last-level cache.  Cached loads while H fits it (H then
// stays there from step to step), nontemporal loads beyond: N = 4096 (68 MB)
// 4% faster cached, M = 7808 (244 MB) 38.3 vs 43.8 us, N = 16384 (1.07 GB)
// 189.7 us nontemporal vs 204.1 cached.  32-frequency Gram stages up to half
// the cache, 16 beyond: N = 4096 124 vs 131 us, M = 7808 395 vs 404 us,
// N = 16384 3.43 vs 3.61 ms.
constexpr size_t kLlcBytes = size_t(256) << 20;
constexpr int kGramKBSmall = 32, kGramKBLarge = 16;

// Largest number of frequencies per pulse.
constexpr int kMaxFreq = 1024;

// Rows of the stacked operator per partial-row chunk of the store-all
// comparator.
constexpr int kStoreRows = 64;

// Bytes of the device vector types the layout counts (complex64 = float2,
// float4, double2, int2); the HIP sources check them against the real types.
constexpr size_t kBytesC64 = 8;
constexpr size_t kBytesF4 = 16;
constexpr size_t kBytesD2 = 16;
constexpr size_t kBytesI2 = 8;

// Scalars that live on the device because they depend on data.
struct DevScalars {
  double lam;           // l1 weight
  double L;             // L_n
  double tau;           // 1 / L_n
  double alpha;         // lam * tau, the shrink threshold
  double sigma2;        // ||A_s||_2^2 of the last pushed pulse
  double rho;           // Rayleigh quotient of the last FISTA step before the last push
  unsigned dbmax_bits;  // max_i |Delta b_i| of the first pulse, float bits
  unsigned fault;       // != 0: a grid barrier of the resident step kernel timed out
  double sig2_acc;      // sum of sigma^2 of the pulses pushed since that step
  double pad1;
};

// One FISTA work item: tile row I, tiles J0 .. J1-1 (J0 >= I).  Tile (I, J)
// sits at packed index toff + J (toff = index of (I, I) minus I), carried in
// the item so the kernels need no second table lookup before loading H.
struct WorkItem {
  int I, J0, J1, toff;
};

// Most frequency pieces one split remainder tile of the FP32 Gram update is
// cut into (the fix-up kernel holds them all in registers).
constexpr int kGramSplitMaxParts = 8;

constexpr size_t kAlign = 256;
constexpr int kBarStride = 32;  // u32 between the grid-barrier counters (128 bytes)
size_t align_up(size_t x);

struct Layout {
  // N: coefficient count M (length of b, c, ...); npix: pixels
  int N = 0, Npad = 0, nb = 0, K = 0, npos = 0, chunk = 4, nparts = 0, npix = 0;
  size_t nnz = 0;  // edgelet: total pixels over all atoms
  bool has_bp = false;
  size_t bp = 0, counter = 0;
  size_t bar = 0;  // the 8 grid-barrier counters of the resident step kernel
  // store-all comparator: capacity, stacked rows, partial rows
  bool store = false;
  int store_cap = 0, store_chunks = 0;
  size_t Gst = 0, Dst = 0, Ust = 0, Pst = 0;
  // split-BF16 Gram over 2 x 2 tile blocks (large N)
  size_t bf_blocks = 0, nbf_blocks = 0;
  size_t atom_ptr = 0, atom_pix = 0, pix_ptr = 0, pix_atom = 0;
  size_t ntiles = 0, ntiles_grid = 0, nitems = 0;
  // FP32 Gram remainder split: split tiles, pieces per tile, launch grid
  size_t gsplit = 0, gram_grid = 0, gP = 0, gsplit_ij = 0;
  int gparts = 0;
  int gram_kb = kGramKBSmall;  // frequencies per LDS stage of the FP32 Gram update
  bool h_cached = true;        // the tile pass reads H with cached loads
  bool slot_nt = false;        // the tile pass writes its slots with nontemporal stores
  // byte offsets
  size_t H, A, b, c0, c1, z0, z1, w0, w1, Q, slot0, slot1, scal, pos,
      sig2, gtoep, tile_ij, tile_row0, items, echo_tmp, Ahi, Alo;
  // differentiation form (record_every > 0)
  int rec_every = 0, rec_pulses = 0, rec_iters = 0, n_ckpt = 0;
  size_t state_bytes = 0;
  size_t ckpt = 0, pulses_d = 0, seg_H = 0, seg_u = 0, seg_db = 0, seg_scal = 0, chat_bar = 0,
         ubar0 = 0, ubar1 = 0, cpart0 = 0, cpart1 = 0, bbar = 0, Bbar = 0, alpha_parts = 0,
         lam_dev = 0, phase_dev = 0;
  size_t total = 0;
};

size_t state_record_bytes(const Layout &L);
size_t count_items(int nb, int chunk);
// Edgelet atoms of the dictionary (rule in include/ofista.h): pixel lists in
// atom order; the atom count, or -1 when a length is out of range.
long long edgelet_atoms(const ofista_config *c, std::vector<int> *ptr, std::vector<int> *pix);
// Coefficient count and total atom pixels for a checked config.
long long coef_count(const ofista_config *c, size_t *nnz);
// OFISTA_OK or the status ofista_create would return for cfg (workspace
// aside), with the reason in *why when given.
ofista_status check(const ofista_config *c, std::string *why);
Layout layout(const ofista_config *c);
const char *status_text(ofista_status st);

}  // namespace ofista
