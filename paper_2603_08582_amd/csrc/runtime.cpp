// Host runtime of libofista: configuration checks, workspace layout, the
// per-pulse launch sequence and the C ABI declared in include/ofista.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ofista.h"
#include "ofista_internal.h"

using namespace ofista;

// Matvec partials of ofista_reconstruct_static: a fixed array in device
// memory, one instance per GPU, alive until the process ends.  Host code never
// passes the array's name to a kernel (it is a host-side stand-in there); it
// uses the device address hipGetSymbolAddress returns for the current device.
static constexpr size_t kStaticScratchBytes = size_t{16} << 20;  // nb <= 128 tile rows
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, resolved once.
hipError_t static_scratch(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

enum ProfClass {
  kProfGram = 0,
  kProfStep = 1,
  kProfRows = 2,
  kProfCorr = 3,
  kProfScalars = 4,
  kProfUpdate = 5,
  kProfStoreFwd = 6,
  kProfStoreAdj = 7,
  kProfResident = 8,
  kProfN = 9
};

}  // namespace

struct ofista_ctx {
  ofista_config cfg{};
  Layout L;
  Geom g{};
  DictTabs dt{};
  // store-all comparator buffers (NULL in the Gram mode)
  float2 *Gst = nullptr, *Dst = nullptr;
  const int2 *bf_blocks = nullptr;  // split-BF16 block table (large N), else NULL
  float2 *gP = nullptr;              // FP32 Gram remainder pieces (else NULL)
  const int2 *gsplit_ij = nullptr;   // (I, J) of the split tiles
  float4 *Ust = nullptr, *Pst = nullptr;
  DevState d{};
  hipStream_t st = nullptr;
  int device = 0;
  int res_grid = 0;       // workgroups of the resident step kernel (0: not available)
  uint64_t bar_gen = 0;   // grid barriers completed since the counters were zeroed
  bool poisoned = false;
  hipError_t hip_err = hipSuccess;
  std::string msg;
  // static detail for a non-HIP status of the last call (no allocation)
  const char *note = nullptr;
  ofista_status note_st = OFISTA_OK;
  // host-side state (all data independent)
  int64_t n = 0;       // pulses since reset
  int64_t G = 0;       // FISTA steps since reset
  bool have_iter = false;
  bool step_since_push = false;  // a FISTA step ran after the last push
  double t = 1.0;
  // differentiation form: what was pushed, and the segment being re-run
  struct PulseRec {
    int s;
    double phase;
    int iters;       // -1: no reconstruct followed this push
    double t_start;  // momentum scalar at the start of that reconstruct
  };
  std::vector<PulseRec> rec;
  char *base = nullptr;  // workspace
  // profiling
  bool prof = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  std::vector<hipEvent_t> pool;
};

namespace {

ofista_status fail_hip(ofista_ctx *c, hipError_t e, const char *where) {
  c->poisoned = true;
  c->hip_err = e;
  c->msg = std::string(where) + ": " + hipGetErrorString(e);
  return OFISTA_E_HIP;
}

#define OF_CK(ctx, expr)                                      \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, #expr); \
  } while (0)

ofista_status usable(ofista_ctx *c) {
  if (!c) return OFISTA_E_ARG;
  if (c->poisoned) return OFISTA_E_STATE;
  return OFISTA_OK;
}

hipEvent_t take_event(ofista_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one launch with events when profiling.
// Events around one launch when profiling.  A scope made with attach = true
// records nothing itself: its events go to the launcher, which has the
// runtime stamp them at the start and end of that kernel (t0(), t1()).
struct ProfScope {
  ofista_ctx *c;
  int cls;
  bool attach;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(ofista_ctx *ctx, int k, bool attach_to_kernel = false)
      : c(ctx), cls(k), attach(attach_to_kernel) {
    if (c->prof) {
      a = take_event(c);
      b = take_event(c);
      if (a && b && !attach) hipEventRecord(a, c->st);
    }
  }
  hipEvent_t t0() const { return a && b ? a : nullptr; }
  hipEvent_t t1() const { return a && b ? b : nullptr; }
  ~ProfScope() {
    if (c->prof && a && b) {
      if (!attach) hipEventRecord(b, c->st);
      c->ev.push_back({cls, {a, b}});
    }
  }
};

ofista_status do_reset(ofista_ctx *c) {
  const Layout &L = c->L;
  const DevState &d = c->d;
  const size_t vecw = static_cast<size_t>(L.Npad) * 2;  // u32 words per vector
  OF_CK(c, launch_fill(d.H, L.ntiles * kTile * kTile * 2, 0u, c->st));
  OF_CK(c, launch_fill(d.b, vecw, 0u, c->st));
  for (int p = 0; p < 2; ++p) {
    OF_CK(c, launch_fill(d.cbuf[p], vecw, 0u, c->st));
    OF_CK(c, launch_fill(d.zbuf[p], vecw, 0u, c->st));
  }
  OF_CK(c, launch_fill(d.wbuf[1], vecw, 0u, c->st));
  OF_CK(c, launch_fill(d.scal, sizeof(DevScalars) / 4, 0u, c->st));
  OF_CK(c, launch_fill(d.bar, 8 * kBarStride, 0u, c->st));
  c->bar_gen = 0;
  if (d.bp) OF_CK(c, launch_fill(d.bp, static_cast<size_t>(L.npix) * 2, 0u, c->st));
  OF_CK(c, launch_init_power(d.wbuf[0], d.slots[0], d.slots[1], L.N, L.Npad, L.nparts, c->st));
  c->n = 0;
  c->G = 0;
  c->have_iter = false;
  c->step_since_push = false;
  c->t = 1.0;
  c->rec.clear();
  return OFISTA_OK;
}

}  // namespace

extern "C" {

ofista_status ofista_create(const ofista_config *cfg, void *d_workspace, size_t ws_bytes,
                            void *hip_stream, ofista_ctx **out) {
  if (!out) return OFISTA_E_ARG;
  *out = nullptr;
  ofista_status st = check(cfg, nullptr);
  if (st != OFISTA_OK) return st;
  const Layout L = layout(cfg);
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0 ||
      ws_bytes < L.total)
    return OFISTA_E_WORKSPACE;
  ofista_ctx *c = new (std::nothrow) ofista_ctx();
  if (!c) return OFISTA_E_ARG;
  c->cfg = *cfg;
  c->cfg.pos_xyz = nullptr;  // host tables are not kept
  c->cfg.edge_lengths = nullptr;
  c->cfg.edge_rotations_deg = nullptr;
  c->L = L;
  c->st = static_cast<hipStream_t>(hip_stream);
  Geom &g = c->g;
  g.nx = cfg->n_x;
  g.ny = cfg->n_y;
  g.N = L.N;
  g.Npad = L.Npad;
  g.K = L.K;
  g.npos = L.npos;
  g.npix = L.npix;
  g.x0 = cfg->x0;
  g.y0 = cfg->y0;
  g.dx = cfg->dx;
  g.dy = cfg->dy;
  g.f0 = cfg->freq0_hz;
  g.df = cfg->dfreq_hz;

  char *base = static_cast<char *>(d_workspace);
  c->base = base;
  DevState &d = c->d;
  d.H = reinterpret_cast<float2 *>(base + L.H);
  d.A = reinterpret_cast<float2 *>(base + L.A);
  d.b = reinterpret_cast<float2 *>(base + L.b);
  d.cbuf[0] = reinterpret_cast<float2 *>(base + L.c0);
  d.cbuf[1] = reinterpret_cast<float2 *>(base + L.c1);
  d.zbuf[0] = reinterpret_cast<float2 *>(base + L.z0);
  d.zbuf[1] = reinterpret_cast<float2 *>(base + L.z1);
  d.wbuf[0] = reinterpret_cast<float2 *>(base + L.w0);
  d.wbuf[1] = reinterpret_cast<float2 *>(base + L.w1);
  d.Q = reinterpret_cast<float4 *>(base + L.Q);
  d.slots[0] = reinterpret_cast<double *>(base + L.slot0);
  d.slots[1] = reinterpret_cast<double *>(base + L.slot1);
  d.scal = reinterpret_cast<DevScalars *>(base + L.scal);
  d.pos = reinterpret_cast<double *>(base + L.pos);
  d.sig2 = reinterpret_cast<double *>(base + L.sig2);
  d.gtoep = reinterpret_cast<double2 *>(base + L.gtoep);
  d.tile_ij = reinterpret_cast<int2 *>(base + L.tile_ij);
  d.tile_row0 = reinterpret_cast<int *>(base + L.tile_row0);
  d.items = reinterpret_cast<WorkItem *>(base + L.items);
  d.echo_tmp = reinterpret_cast<double2 *>(base + L.echo_tmp);
  d.Ahi = L.Ahi ? reinterpret_cast<unsigned *>(base + L.Ahi) : nullptr;
  d.Alo = L.Alo ? reinterpret_cast<unsigned *>(base + L.Alo) : nullptr;
  const bool edgelet = cfg->dict == OFISTA_DICT_EDGELET;
  d.atom_ptr = edgelet ? reinterpret_cast<int *>(base + L.atom_ptr) : nullptr;
  d.atom_pix = edgelet ? reinterpret_cast<int *>(base + L.atom_pix) : nullptr;
  d.pix_ptr = edgelet ? reinterpret_cast<int *>(base + L.pix_ptr) : nullptr;
  d.pix_atom = edgelet ? reinterpret_cast<int *>(base + L.pix_atom) : nullptr;
  c->dt = DictTabs{cfg->dict, cfg->haar_levels, d.atom_ptr, d.atom_pix, d.pix_ptr, d.pix_atom};
  d.counter = reinterpret_cast<unsigned *>(base + L.counter);
  d.bar = reinterpret_cast<unsigned *>(base + L.bar);
  d.bp = L.has_bp ? reinterpret_cast<float2 *>(base + L.bp) : nullptr;
  c->Gst = L.store ? reinterpret_cast<float2 *>(base + L.Gst) : nullptr;
  c->Dst = L.store ? reinterpret_cast<float2 *>(base + L.Dst) : nullptr;
  c->Ust = L.store ? reinterpret_cast<float4 *>(base + L.Ust) : nullptr;
  c->Pst = L.store ? reinterpret_cast<float4 *>(base + L.Pst) : nullptr;

  // host tables
  const int nb = L.nb;
  std::vector<int2> tij(std::max(L.ntiles_grid, L.gram_grid), make_int2(-1, -1));
  std::vector<int2> split_ij;
  std::vector<int> row0(nb);
  {
    // storage order: row-major upper tiles
    size_t t = 0;
    for (int I = 0; I < nb; ++I) {
      row0[I] = static_cast<int>(t);
      t += static_cast<size_t>(nb - I);
    }
    // Gram launch order: 8 x 8 super-tiles of the upper triangle, row-major
    // over super-tiles, so that a run of the table touches few A blocks
    t = 0;
    constexpr int S = 8;
    const int ns = L.store ? 0 : (nb + S - 1) / S;  // no Gram when storing pulses
    for (int P = 0; P < ns; ++P)
      for (int Qs = P; Qs < ns; ++Qs)
        for (int I = P * S; I < std::min(nb, P * S + S); ++I)
          for (int J = std::max(I, Qs * S); J < std::min(nb, Qs * S + S); ++J) tij[t++] = make_int2(I, J);
    if (L.gsplit > 0) {
      // The last gsplit off-diagonal tiles of that order are split.  XCD x
      // (workgroups b = x mod 8) reads the table chunk [x per, (x+1) per):
      // its eighth of the whole tiles, then the pieces k = x mod 8.
      const std::vector<int2> ord(tij.begin(), tij.begin() + L.ntiles);
      std::vector<char> cut(L.ntiles, 0);
      for (size_t u = L.ntiles; u-- > 0 && split_ij.size() < L.gsplit;)
        if (ord[u].x != ord[u].y) {
          cut[u] = 1;
          split_ij.push_back(ord[u]);
        }
      std::reverse(split_ij.begin(), split_ij.end());
      std::vector<int2> whole, pieces;
      for (size_t u = 0; u < L.ntiles; ++u)
        if (!cut[u]) whole.push_back(ord[u]);
      for (size_t sidx = 0; sidx < split_ij.size(); ++sidx)
        for (int p = 1; p <= L.gparts; ++p)
          pieces.push_back(make_int2(split_ij[sidx].x | static_cast<int>(sidx << 16),
                                     split_ij[sidx].y | (p << 20)));
      const size_t per = L.gram_grid / 8, wper = whole.size() / 8;
      std::fill(tij.begin(), tij.end(), make_int2(-1, -1));
      for (size_t x = 0; x < 8; ++x) {
        size_t o = x * per;
        for (size_t u = 0; u < wper; ++u) tij[o++] = whole[x * wper + u];
        for (size_t k = x; k < pieces.size(); k += 8) tij[o++] = pieces[k];
      }
    }
  }
  std::vector<int2> bfb;
  if (L.nbf_blocks) {
    // 8 x 8 super-blocks, row-major over super-blocks; launch block b runs on
    // XCD b % 8, so entry b of the table is list entry (b % 8) per + b / 8:
    // each XCD works through a contiguous run of the list, and its ~64
    // concurrent blocks (about one super-block) use 32 panels
    const int nbB = (nb + 1) / 2, S = 8, ns = (nbB + S - 1) / S;
    std::vector<int2> list;
    list.reserve(L.nbf_blocks);
    for (int P = 0; P < ns; ++P)
      for (int Qs = P; Qs < ns; ++Qs)
        for (int IB = P * S; IB < std::min(nbB, P * S + S); ++IB)
          for (int JB = std::max(IB, Qs * S); JB < std::min(nbB, Qs * S + S); ++JB)
            list.push_back(make_int2(IB, JB));
    const size_t per = L.nbf_blocks / 8;
    bfb.assign(L.nbf_blocks, make_int2(-1, -1));
    for (size_t b = 0; b < L.nbf_blocks; ++b) {
      const size_t k = (b % 8) * per + b / 8;
      if (k < list.size()) bfb[b] = list[k];
    }
    c->bf_blocks = reinterpret_cast<const int2 *>(base + L.bf_blocks);
  }
  if (L.gsplit > 0) {
    c->gP = reinterpret_cast<float2 *>(base + L.gP);
    c->gsplit_ij = reinterpret_cast<const int2 *>(base + L.gsplit_ij);
  }
  // Full runs first, then the short last runs of the rows: the short items
  // then fill the tail of the pass instead of delaying full ones (-3% at
  // N = 4096, neutral at 16384).  Slots depend on (I, J0) only, so the order
  // does not change any result.
  std::vector<WorkItem> items;
  items.reserve(L.nitems);
  for (int I = 0; I < nb; ++I)
    for (int J0 = I; J0 < nb; J0 += L.chunk)
      items.push_back(WorkItem{I, J0, J0 + L.chunk < nb ? J0 + L.chunk : nb, row0[I] - I});
  std::stable_partition(items.begin(), items.end(),
                        [&](const WorkItem &w) { return w.J1 - w.J0 == L.chunk; });

  auto fail = [&](hipError_t e, const char *where) {
    fail_hip(c, e, where);
    *out = c;  // hand back the poisoned ctx so the caller can read the message
    return OFISTA_E_HIP;
  };
  hipError_t e;
  if ((e = hipGetDevice(&c->device)) != hipSuccess) return fail(e, "hipGetDevice");
  {
    int n_cu = 0;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device)) !=
        hipSuccess)
      return fail(e, "hipDeviceGetAttribute");
    // AUTO runs the launch pair: at N = 4096 on MI355X it measured 17.6 us
    // per step against 26 us for the resident kernel
    if (cfg->step_kernel == OFISTA_STEP_RESIDENT && !L.store) c->res_grid = resident_grid(c->device, n_cu);
    // the resident kernel stages z, w per work item and sums the update
    // parts in registers: bounded counts of both
    if (L.nitems > static_cast<size_t>(kResMaxItems) * c->res_grid || L.nparts > kResMaxParts)
      c->res_grid = 0;
    if (cfg->step_kernel == OFISTA_STEP_RESIDENT && c->res_grid == 0) {
      c->note = "ofista_create: the resident step kernel needs cooperative launch and at most "
                "5 work items per CU";
      c->note_st = OFISTA_E_UNSUPPORTED;
      *out = c;
      return OFISTA_E_UNSUPPORTED;
    }
  }
  {
    void *sp = nullptr;  // per-device static partials (ofista_reconstruct_static)
    if ((e = static_scratch(c->device, &sp)) != hipSuccess) return fail(e, "hipGetSymbolAddress");
  }
  if ((e = hipMemcpyAsync(d.pos, cfg->pos_xyz, 3 * sizeof(double) * L.npos, hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy positions");
  if (!tij.empty() &&
      (e = hipMemcpyAsync(d.tile_ij, tij.data(), tij.size() * sizeof(int2), hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy tile table");
  if ((e = hipMemcpyAsync(d.tile_row0, row0.data(), row0.size() * sizeof(int), hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy tile rows");
  if (!bfb.empty() &&
      (e = hipMemcpyAsync(const_cast<int2 *>(c->bf_blocks), bfb.data(), bfb.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy block table");
  if ((e = hipMemcpyAsync(d.items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy work items");
  if (!split_ij.empty() &&
      (e = hipMemcpyAsync(const_cast<int2 *>(c->gsplit_ij), split_ij.data(), split_ij.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->st)) != hipSuccess)
    return fail(e, "copy split tiles");
  std::vector<int> aptr, apix, pptr, patom;
  if (edgelet) {
    edgelet_atoms(cfg, &aptr, &apix);
    // pixel -> atoms, atoms in increasing order
    pptr.assign(static_cast<size_t>(L.npix) + 1, 0);
    for (int q : apix) ++pptr[static_cast<size_t>(q) + 1];
    for (int p = 0; p < L.npix; ++p) pptr[p + 1] += pptr[p];
    patom.assign(apix.size(), 0);
    std::vector<int> fill(pptr.begin(), pptr.end() - 1);
    for (int m = 0; m < L.N; ++m)
      for (int q = aptr[m]; q < aptr[m + 1]; ++q) patom[fill[apix[q]]++] = m;
    if ((e = hipMemcpyAsync(d.atom_ptr, aptr.data(), aptr.size() * sizeof(int), hipMemcpyHostToDevice, c->st)) != hipSuccess ||
        (e = hipMemcpyAsync(d.atom_pix, apix.data(), apix.size() * sizeof(int), hipMemcpyHostToDevice, c->st)) != hipSuccess ||
        (e = hipMemcpyAsync(d.pix_ptr, pptr.data(), pptr.size() * sizeof(int), hipMemcpyHostToDevice, c->st)) != hipSuccess ||
        (e = hipMemcpyAsync(d.pix_atom, patom.data(), patom.size() * sizeof(int), hipMemcpyHostToDevice, c->st)) != hipSuccess)
      return fail(e, "copy edgelet tables");
    // sigma^2 per position from the K x K FP64 matrix A_s A_s^H, in batches
    // that fit the (not yet used) H region
    const size_t per = static_cast<size_t>(L.K) * L.K;
    const size_t scratch = L.store ? static_cast<size_t>(L.store_cap) * L.K * L.Npad * sizeof(float2)
                                   : L.ntiles * kTile * kTile * sizeof(float2);
    const size_t batch = std::max<size_t>(1, scratch / (per * sizeof(double2)));
    double2 *Gs = reinterpret_cast<double2 *>(L.store ? base + L.Gst : reinterpret_cast<char *>(d.H));
    for (int s0 = 0; s0 < L.npos; s0 += static_cast<int>(batch)) {
      const int nm = static_cast<int>(std::min<size_t>(batch, static_cast<size_t>(L.npos - s0)));
      for (int j = 0; j < nm; ++j) {
        if ((e = launch_rows(g, d.pos, s0 + j, d.A, c->dt, c->st)) != hipSuccess ||
            (e = launch_gram_kk(g, d.A, Gs + static_cast<size_t>(j) * per, c->st)) != hipSuccess)
          return fail(e, "sigma2 rows");
      }
      if ((e = launch_sigma2_dense(L.K, Gs, nm, d.sig2 + s0, c->st)) != hipSuccess)
        return fail(e, "sigma2 eigenvalue");
    }
  } else if ((e = launch_sigma2(g, d.pos, d.gtoep, d.sig2, c->st)) != hipSuccess) {
    return fail(e, "sigma2 kernels");
  }
  st = do_reset(c);
  if (st != OFISTA_OK) {
    *out = c;
    return st;
  }
  if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return fail(e, "hipStreamSynchronize");
  *out = c;
  return OFISTA_OK;
}

ofista_status ofista_reset(ofista_ctx *c) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  return do_reset(c);
}

}  // extern "C"

namespace {

float2 *seg_ptr(ofista_ctx *c, size_t off, size_t idx, size_t stride) {
  return reinterpret_cast<float2 *>(c->base + off + idx * stride);
}

// One pulse: rows, H and b updates, scalars.  seg_j >= 0 while the backward
// pass re-runs pulse seg_j of a segment: then also keep H_n, Delta b_n and the
// scalars of this pulse.
ofista_status push_store(ofista_ctx *c, const void *d_pulse, int32_t s, double phase_corr);

ofista_status push_impl(ofista_ctx *c, const void *d_pulse, int32_t s, double phase_corr, int seg_j) {
  if (c->L.store) return push_store(c, d_pulse, s, phase_corr);
  const DevState &d = c->d;
  const Layout &L = c->L;
  const int first = c->n == 0 ? 1 : 0;
  const int par = static_cast<int>(c->G & 1);
  const ScalarArgs sca{d.scal, d.sig2, d.slots[par], d.slots[par ^ 1], c->cfg.lambda, s, first,
                       c->cfg.lambda_relative, c->cfg.lipschitz, c->step_since_push ? 1 : 0,
                       L.nparts};
  bool scal_done = false;
  {
    ProfScope p(c, kProfRows);
    OF_CK(c, launch_rows(c->g, d.pos, s, d.A, c->dt, c->st));
  }
  if (d.bp)
    OF_CK(c, launch_backproject(c->g, d.pos, s, static_cast<const float2 *>(d_pulse),
                                std::cos(phase_corr), std::sin(phase_corr), d.bp, c->st));
  if (seg_j >= 0) {
    OF_CK(c, launch_corr(c->g, d.A, static_cast<const float2 *>(d_pulse), std::cos(phase_corr),
                         std::sin(phase_corr), nullptr, d.scal, 0, c->st,
                         seg_ptr(c, L.seg_db, seg_j, static_cast<size_t>(L.Npad) * sizeof(float2))));
  }
  if (c->cfg.precision == OFISTA_PREC_SPLIT_BF16) {
    {
      ProfScope p(c, kProfCorr);
      OF_CK(c, launch_corr(c->g, d.A, static_cast<const float2 *>(d_pulse), std::cos(phase_corr),
                           std::sin(phase_corr), d.b, d.scal, first, c->st));
    }
    ProfScope p(c, kProfGram, true);
    OF_CK(c, launch_gram_bf16x3(c->g, d.A, d.Ahi, d.Alo, d.H, d.tile_ij,
                                static_cast<int>(L.ntiles_grid), c->bf_blocks,
                                static_cast<int>(L.nbf_blocks), c->st, p.t0(), p.t1()));
  } else {
    ProfScope p(c, kProfGram, true);
    CorrArgs corr{static_cast<const float2 *>(d_pulse), static_cast<float>(std::cos(phase_corr)),
                  static_cast<float>(std::sin(phase_corr)), d.b, d.scal, first};
    const GramSplit split{c->gP, c->gsplit_ij, static_cast<int>(L.gsplit), L.gparts};
    OF_CK(c, launch_gram_fp32(c->g, d.A, d.H, d.tile_ij, static_cast<int>(L.gram_grid), corr, split,
                              L.gram_kb, &sca, &scal_done, c->st, p.t0(), p.t1()));
  }
  if (!scal_done) {  // else the Gram fix-up launch ran them
    ProfScope p(c, kProfScalars);
    OF_CK(c, launch_scalars(sca, c->st));
  }
  c->step_since_push = false;
  if (seg_j >= 0) {
    const size_t hbytes = L.ntiles * kTile * kTile * sizeof(float2);
    OF_CK(c, hipMemcpyAsync(c->base + L.seg_H + seg_j * hbytes, d.H, hbytes, hipMemcpyDeviceToDevice,
                            c->st));
    OF_CK(c, hipMemcpyAsync(c->base + L.seg_scal + seg_j * sizeof(DevScalars), d.scal,
                            sizeof(DevScalars), hipMemcpyDeviceToDevice, c->st));
  }
  c->n += 1;
  return OFISTA_OK;
}

// Store-all comparator: keep G_s = F_s W and the rotated data of pulse n in
// slot n; lambda from Delta b_1 = G_1^H d~_1 (the correlation kernel with no
// b), then the same scalars as the Gram mode.  b stays zero: the gradient
// sum_k G_k^H (G_k z - d_k) already holds the data term.
ofista_status push_store(ofista_ctx *c, const void *d_pulse, int32_t s, double phase_corr) {
  const DevState &d = c->d;
  const Layout &L = c->L;
  if (c->n >= L.store_cap) return OFISTA_E_STATE;
  const int first = c->n == 0 ? 1 : 0;
  float2 *G = c->Gst + static_cast<size_t>(c->n) * L.K * L.Npad;
  {
    ProfScope p(c, kProfRows);
    OF_CK(c, launch_rows(c->g, d.pos, s, G, c->dt, c->st));
  }
  if (d.bp)
    OF_CK(c, launch_backproject(c->g, d.pos, s, static_cast<const float2 *>(d_pulse),
                                std::cos(phase_corr), std::sin(phase_corr), d.bp, c->st));
  OF_CK(c, launch_rotate(static_cast<const float2 *>(d_pulse), L.K, std::cos(phase_corr),
                         std::sin(phase_corr), c->Dst + static_cast<size_t>(c->n) * L.K, c->st));
  if (first)
    OF_CK(c, launch_corr(c->g, G, static_cast<const float2 *>(d_pulse), std::cos(phase_corr),
                         std::sin(phase_corr), nullptr, d.scal, 1, c->st));
  {
    ProfScope p(c, kProfScalars);
    const int par = static_cast<int>(c->G & 1);
    const ScalarArgs sca{d.scal, d.sig2, d.slots[par], d.slots[par ^ 1], c->cfg.lambda, s, first,
                         c->cfg.lambda_relative, c->cfg.lipschitz, c->step_since_push ? 1 : 0,
                         L.nparts};
    OF_CK(c, launch_scalars(sca, c->st));
    c->step_since_push = false;
  }
  c->n += 1;
  return OFISTA_OK;
}

// Algorithm 1 with `iters` steps; seg_j >= 0 also keeps u of every step.
ofista_status reconstruct_impl(ofista_ctx *c, int32_t iters, void *d_coef_out, int seg_j,
                               double *t_start_out, float4 *Q = nullptr) {
  const DevState &d = c->d;
  const Layout &L = c->L;
  double t = (c->n == 1 || c->cfg.momentum == OFISTA_MOMENTUM_RESTART) ? 1.0 : c->t;
  if (t_start_out) *t_start_out = t;
  const bool resident = c->res_grid > 0 && !L.store && seg_j < 0;
  for (int k0 = 0; resident && k0 < iters; k0 += kResMaxSteps) {
    ResidentArgs a{};
    a.H = d.H;
    a.items = d.items;
    a.b = d.b;
    for (int p = 0; p < 2; ++p) {
      a.zbuf[p] = d.zbuf[p];
      a.cbuf[p] = d.cbuf[p];
      a.wbuf[p] = d.wbuf[p];
      a.slots[p] = d.slots[p];
    }
    a.Q = Q ? Q : d.Q;
    a.scal = d.scal;
    a.bar = d.bar;
    a.nb = L.nb;
    a.N = L.N;
    a.nitems = static_cast<int>(L.nitems);
    a.nparts = L.nparts;
    a.p0 = static_cast<int>(c->G & 1);
    a.iters = std::min(kResMaxSteps, iters - k0);
    a.warm = k0 == 0;
    for (int k = 0; k < a.iters; ++k) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      a.beta[k] = static_cast<float>(c->cfg.momentum == OFISTA_MOMENTUM_ISTA ? 0.0 : (t - 1.0) / tn);
      t = tn;
    }
    if (c->bar_gen + 2 * kResMaxSteps > (1u << 24)) {  // keep the counters far from wrapping
      OF_CK(c, launch_fill(d.bar, 8 * kBarStride, 0u, c->st));
      c->bar_gen = 0;
    }
    a.bar_gen = static_cast<unsigned>(c->bar_gen);
    {
      ProfScope ps(c, kProfResident);
      OF_CK(c, launch_steps_resident(a, c->res_grid, c->st));
    }
    c->bar_gen += 2 * static_cast<uint64_t>(a.iters);
    c->G += a.iters;
  }
  for (int k = 0; !resident && k < iters; ++k) {
    const int p = static_cast<int>(c->G & 1);
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double beta = c->cfg.momentum == OFISTA_MOMENTUM_ISTA ? 0.0 : (t - 1.0) / tn;
    StepArgs a{};
    a.H = d.H;
    a.zc = k == 0 ? d.cbuf[p] : d.zbuf[p];
    a.wc = d.wbuf[p];
    a.b = d.b;
    a.cc = d.cbuf[p];
    a.cn = d.cbuf[p ^ 1];
    a.zn = d.zbuf[p ^ 1];
    a.wn = d.wbuf[p ^ 1];
    a.Q = Q ? Q : d.Q;
    a.slot_prev = d.slots[p];
    a.slot_cur = d.slots[p ^ 1];
    a.scal = d.scal;
    a.items = d.items;
    a.urec = seg_j >= 0 ? seg_ptr(c, L.seg_u, static_cast<size_t>(seg_j) * L.rec_iters + k,
                                  static_cast<size_t>(L.Npad) * sizeof(float2))
                        : nullptr;
    a.nb = L.nb;
    a.N = L.N;
    a.nitems = static_cast<int>(L.nitems);
    a.chunk = L.chunk;
    a.h_cached = L.h_cached;
    a.slot_nt = L.slot_nt;
    a.beta = static_cast<float>(beta);
    if (L.store) {
      // gradient from the n stored pulses: two passes over the stacked rows
      const int rows = static_cast<int>(c->n) * L.K;
      a.P = c->Pst;
      a.nchunks = (rows + kStoreRows - 1) / kStoreRows;
      a.Npad = L.Npad;
      {
        ProfScope ps(c, kProfStoreFwd, true);
        OF_CK(c, launch_store_forward(c->Gst, c->Dst, rows, L.Npad, L.N, a.zc, a.wc, c->Ust, c->st,
                                      ps.t0(), ps.t1()));
      }
      {
        ProfScope ps(c, kProfStoreAdj, true);
        OF_CK(c, launch_store_adjoint(c->Gst, rows, L.Npad, c->Ust, c->Pst, c->st, ps.t0(), ps.t1()));
      }
    } else {
      ProfScope ps(c, kProfStep, true);
      OF_CK(c, launch_step_tiles(a, c->st, ps.t0(), ps.t1()));
    }
    {
      ProfScope ps(c, kProfUpdate, true);
      OF_CK(c, launch_step_update(a, c->st, ps.t0(), ps.t1()));
    }
    c->G += 1;
    t = tn;
  }
  c->t = t;
  if (iters > 0) c->have_iter = c->step_since_push = true;
  if (d_coef_out) {
    OF_CK(c, hipMemcpyAsync(d_coef_out, d.cbuf[c->G & 1], static_cast<size_t>(L.N) * sizeof(float2),
                            hipMemcpyDeviceToDevice, c->st));
  }
  return OFISTA_OK;
}

ofista_status export_to(ofista_ctx *c, void *d_buf);
ofista_status import_from(ofista_ctx *c, const void *d_buf);

}  // namespace

extern "C" {

ofista_status ofista_push_pulse(ofista_ctx *c, const void *d_pulse, int32_t s, double phase_corr) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_pulse || !std::isfinite(phase_corr)) return OFISTA_E_ARG;
  if (s < 0 || s >= c->L.npos) return OFISTA_E_RANGE;
  const Layout &L = c->L;
  if (c->cfg.validate_input) {
    unsigned bad = 0;
    OF_CK(c, launch_count_nonfinite(static_cast<const float2 *>(d_pulse), L.K, c->d.counter, c->st));
    OF_CK(c, hipMemcpyAsync(&bad, c->d.counter, sizeof(unsigned), hipMemcpyDeviceToHost, c->st));
    OF_CK(c, hipStreamSynchronize(c->st));
    if (bad) {
      c->note = "ofista_push_pulse: the pulse holds a non-finite sample (nothing was changed)";
      c->note_st = OFISTA_E_ARG;
      return OFISTA_E_ARG;
    }
  }
  if (L.rec_every > 0) {
    if (c->n >= L.rec_pulses) return OFISTA_E_STATE;  // recording capacity reached
    if (c->n % L.rec_every == 0) {
      st = export_to(c, c->base + L.ckpt + static_cast<size_t>(c->n / L.rec_every) * align_up(L.state_bytes));
      if (st != OFISTA_OK) return st;
    }
    OF_CK(c, hipMemcpyAsync(c->base + L.pulses_d + static_cast<size_t>(c->n) * L.K * sizeof(float2), d_pulse,
                            static_cast<size_t>(L.K) * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
    c->rec.push_back(ofista_ctx::PulseRec{s, phase_corr, -1, 0.0});
  }
  return push_impl(c, d_pulse, s, phase_corr, -1);
}

ofista_status ofista_reconstruct(ofista_ctx *c, int32_t iters, void *d_coef_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (iters < 0) return OFISTA_E_ARG;
  if (c->n == 0) return OFISTA_E_STATE;
  double t0 = 0.0;
  if (c->L.rec_every > 0) {
    if (c->rec.empty() || c->rec.back().iters >= 0) return OFISTA_E_STATE;  // one per pulse
    if (iters > c->L.rec_iters) return OFISTA_E_ARG;
  }
  st = reconstruct_impl(c, iters, d_coef_out, -1, &t0);
  if (st == OFISTA_OK && c->L.rec_every > 0) {
    c->rec.back().iters = iters;
    c->rec.back().t_start = t0;
  }
  return st;
}

ofista_status ofista_reconstruct_static(ofista_ctx *c, int32_t iters, void *d_coef_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  const Layout &L = c->L;
  if (L.store) {
    c->note = "ofista_reconstruct_static: PULSES storage has no matvec partials";
    c->note_st = OFISTA_E_UNSUPPORTED;
    return OFISTA_E_UNSUPPORTED;
  }
  const size_t need = static_cast<size_t>(L.nb) * L.nb * kTile * sizeof(float4);
  if (need > kStaticScratchBytes) {
    c->note = "ofista_reconstruct_static: the matvec partials exceed the 16 MiB static "
              "array (at most 128 tile rows, M <= 8192)";
    c->note_st = OFISTA_E_UNSUPPORTED;
    return OFISTA_E_UNSUPPORTED;
  }
  if (iters < 0) return OFISTA_E_ARG;
  if (c->n == 0) return OFISTA_E_STATE;
  if (c->L.rec_every > 0) {
    if (c->rec.empty() || c->rec.back().iters >= 0) return OFISTA_E_STATE;  // one per pulse
    if (iters > c->L.rec_iters) return OFISTA_E_ARG;
  }
  void *sp = nullptr;  // resolved at create, so this only reads the table
  if (static_scratch(c->device, &sp) != hipSuccess) {
    c->note = "ofista_reconstruct_static: no static array on this device";
    c->note_st = OFISTA_E_STATE;
    return OFISTA_E_STATE;
  }
  // no profiling events here: taking one may create it
  const bool prof = c->prof;
  c->prof = false;
  double t0 = 0.0;
  st = reconstruct_impl(c, iters, d_coef_out, -1, &t0, static_cast<float4 *>(sp));
  c->prof = prof;
  if (st == OFISTA_OK && c->L.rec_every > 0) {
    c->rec.back().iters = iters;
    c->rec.back().t_start = t0;
  }
  return st;
}

ofista_status ofista_set_lambda(ofista_ctx *c, double lam) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!std::isfinite(lam) || lam < 0) return OFISTA_E_ARG;
  c->cfg.lambda = lam;
  c->cfg.lambda_relative = 0;
  OF_CK(c, launch_set_lambda(c->d.scal, lam, c->st));
  return OFISTA_OK;
}

}  // extern "C"

namespace {

// Reverse pass of pulse n (re-run as segment slot j).
ofista_status reverse_pulse(ofista_ctx *c, int n, int j) {
  const Layout &L = c->L;
  const DevState &d = c->d;
  const size_t vbytes = static_cast<size_t>(L.Npad) * sizeof(float2);
  const size_t hbytes = L.ntiles * kTile * kTile * sizeof(float2);
  const ofista_ctx::PulseRec &r = c->rec[n];
  const int m = r.iters < 0 ? 0 : r.iters;
  float2 *ubar[2] = {seg_ptr(c, L.ubar0, 0, 0), seg_ptr(c, L.ubar1, 0, 0)};
  float2 *cpart[2] = {seg_ptr(c, L.cpart0, 0, 0), seg_ptr(c, L.cpart1, 0, 0)};
  double *alpha_parts = reinterpret_cast<double *>(c->base + L.alpha_parts);
  AdjArgs a{};
  a.Q = d.Q;
  a.scal = reinterpret_cast<const DevScalars *>(c->base + L.seg_scal + j * sizeof(DevScalars));
  a.bbar = seg_ptr(c, L.bbar, 0, 0);
  a.chat_bar = seg_ptr(c, L.chat_bar, 0, 0);
  a.Bbar = seg_ptr(c, L.Bbar, 0, 0);
  a.alpha_parts_all = alpha_parts;
  a.nb = L.nb;
  a.N = L.N;
  a.chunk = L.chunk;
  const float2 *dB = seg_ptr(c, L.seg_db, j, vbytes);
  double *lam_out = reinterpret_cast<double *>(c->base + L.lam_dev) + n;
  double *phase_out = reinterpret_cast<double *>(c->base + L.phase_dev) + n;
  if (m == 0) {
    OF_CK(c, launch_fill(a.bbar, static_cast<size_t>(L.Npad) * 2, 0u, c->st));
    OF_CK(c, launch_adj_pulse(a, 0, L.Npad, dB, lam_out, phase_out, c->st));
    return OFISTA_OK;
  }
  // momentum coefficients of the pulse's steps (data independent)
  std::vector<float> beta(m + 1, 0.f);
  {
    double t = r.t_start;
    for (int k = 1; k <= m; ++k) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      beta[k] = c->cfg.momentum == OFISTA_MOMENTUM_ISTA ? 0.f : static_cast<float>((t - 1.0) / tn);
      t = tn;
    }
  }
  auto u_of_step = [&](int k) {  // u_k, k = 1..m
    return seg_ptr(c, L.seg_u, static_cast<size_t>(j) * L.rec_iters + (k - 1), vbytes);
  };
  int cur = 0;
  a.u_prev = u_of_step(m);
  a.ubar_next = ubar[cur];
  a.cpart_next = cpart[cur];
  a.alpha_parts = alpha_parts + static_cast<size_t>(m - 1) * L.nb;
  OF_CK(c, launch_adj_start(a, c->st));
  const float2 *Hn = reinterpret_cast<const float2 *>(c->base + L.seg_H + j * hbytes);
  for (int k = m; k >= 1; --k) {
    StepArgs sa{};
    sa.H = Hn;
    sa.zc = ubar[cur];
    sa.wc = ubar[cur];
    sa.Q = d.Q;
    sa.items = d.items;
    sa.nb = L.nb;
    sa.N = L.N;
    sa.nitems = static_cast<int>(L.nitems);
    sa.chunk = L.chunk;
    sa.h_cached = L.h_cached;
    sa.slot_nt = L.slot_nt;
    OF_CK(c, launch_step_tiles(sa, c->st));
    a.ubar_cur = ubar[cur];
    a.cpart_cur = cpart[cur];
    a.ubar_next = ubar[cur ^ 1];
    a.cpart_next = cpart[cur ^ 1];
    a.last = k == 1 ? 1 : 0;
    a.u_prev = k >= 2 ? u_of_step(k - 1) : nullptr;
    a.alpha_parts = k >= 2 ? alpha_parts + static_cast<size_t>(k - 2) * L.nb : nullptr;
    a.beta_prev = k >= 2 ? beta[k - 1] : 0.f;
    OF_CK(c, launch_adj_update(a, c->st));
    cur ^= 1;
  }
  OF_CK(c, launch_adj_pulse(a, m * L.nb, L.Npad, dB, lam_out, phase_out, c->st));
  return OFISTA_OK;
}

}  // namespace

extern "C" {

ofista_status ofista_backward(ofista_ctx *c, const void *d_grad_img, double *grad_lambda,
                              double *grad_phase) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  const Layout &L = c->L;
  if (L.store) return OFISTA_E_UNSUPPORTED;
  if (L.rec_every <= 0) return OFISTA_E_STATE;
  if (!d_grad_img || !grad_lambda || !grad_phase) return OFISTA_E_ARG;
  const int P = static_cast<int>(c->n);
  if (P == 0 || static_cast<int>(c->rec.size()) != P) return OFISTA_E_STATE;
  const size_t cstride = align_up(L.state_bytes);
  char *final_ckpt = c->base + L.ckpt + static_cast<size_t>(L.n_ckpt - 1) * cstride;
  st = export_to(c, final_ckpt);
  if (st != OFISTA_OK) return st;
  const std::vector<ofista_ctx::PulseRec> rec = c->rec;  // the re-runs below must not record
  OF_CK(c, launch_image_adjoint(c->g, static_cast<const float2 *>(d_grad_img),
                                seg_ptr(c, L.chat_bar, 0, 0), c->dt, c->st));
  OF_CK(c, launch_fill(c->base + L.Bbar, static_cast<size_t>(L.Npad) * 2, 0u, c->st));
  const int R = L.rec_every;
  const int nseg = (P + R - 1) / R;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int n0 = seg * R, n1 = std::min(P, n0 + R);
    st = import_from(c, c->base + L.ckpt + static_cast<size_t>(seg) * cstride);
    if (st != OFISTA_OK) return st;
    for (int n = n0; n < n1; ++n) {
      const void *dn = c->base + L.pulses_d + static_cast<size_t>(n) * L.K * sizeof(float2);
      st = push_impl(c, dn, rec[n].s, rec[n].phase, n - n0);
      if (st != OFISTA_OK) return st;
      if (rec[n].iters >= 0) {
        st = reconstruct_impl(c, rec[n].iters, nullptr, n - n0, nullptr);
        if (st != OFISTA_OK) return st;
      }
    }
    for (int n = n1 - 1; n >= n0; --n) {
      st = reverse_pulse(c, n, n - n0);
      if (st != OFISTA_OK) return st;
    }
  }
  st = import_from(c, final_ckpt);
  if (st != OFISTA_OK) return st;
  c->rec = rec;
  std::vector<double> lam(P), ph(P);
  OF_CK(c, hipStreamSynchronize(c->st));
  OF_CK(c, hipMemcpy(lam.data(), c->base + L.lam_dev, P * sizeof(double), hipMemcpyDeviceToHost));
  OF_CK(c, hipMemcpy(ph.data(), c->base + L.phase_dev, P * sizeof(double), hipMemcpyDeviceToHost));
  double gl = 0.0;
  for (int n = 0; n < P; ++n) {
    gl += lam[n];
    grad_phase[n] = ph[n];
  }
  *grad_lambda = gl;
  return OFISTA_OK;
}

ofista_status ofista_image(ofista_ctx *c, void *d_img_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_img_out) return OFISTA_E_ARG;
  OF_CK(c, launch_image(c->g, c->d.cbuf[c->G & 1], static_cast<float2 *>(d_img_out), c->dt,
                        c->st));
  return OFISTA_OK;
}

ofista_status ofista_vector(ofista_ctx *c, int32_t which, void *d_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_out || which < 0 || which > 2) return OFISTA_E_ARG;
  const float2 *src = which == 0 ? c->d.b : which == 1 ? c->d.cbuf[c->G & 1] : c->d.wbuf[c->G & 1];
  OF_CK(c, hipMemcpyAsync(d_out, src, static_cast<size_t>(c->L.N) * sizeof(float2),
                          hipMemcpyDeviceToDevice, c->st));
  return OFISTA_OK;
}

ofista_status ofista_rows(ofista_ctx *c, int32_t s, void *d_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_out) return OFISTA_E_ARG;
  if (s < 0 || s >= c->L.npos) return OFISTA_E_RANGE;
  OF_CK(c, launch_rows(c->g, c->d.pos, s, c->d.A, c->dt, c->st));
  OF_CK(c, hipMemcpy2DAsync(d_out, static_cast<size_t>(c->L.N) * sizeof(float2), c->d.A,
                            static_cast<size_t>(c->L.Npad) * sizeof(float2),
                            static_cast<size_t>(c->L.N) * sizeof(float2), c->L.K,
                            hipMemcpyDeviceToDevice, c->st));
  return OFISTA_OK;
}

ofista_status ofista_gram(ofista_ctx *c, void *d_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_out) return OFISTA_E_ARG;
  if (c->L.store) return OFISTA_E_UNSUPPORTED;      // no Gram is kept
  if (c->L.N > 16384) return OFISTA_E_UNSUPPORTED;  // inspection of small problems only
  OF_CK(c, launch_gram_dense(c->g, c->d.H, c->d.tile_row0, static_cast<float2 *>(d_out), c->st));
  return OFISTA_OK;
}

ofista_status ofista_gram_entries(ofista_ctx *c, int32_t n, const int32_t *d_i, const int32_t *d_j,
                                  void *d_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (n < 0 || (n > 0 && (!d_i || !d_j || !d_out))) return OFISTA_E_ARG;
  if (c->L.store) return OFISTA_E_UNSUPPORTED;
  OF_CK(c, launch_gram_entries(c->g, c->d.H, c->d.tile_row0, n, d_i, d_j,
                               static_cast<float2 *>(d_out), c->st));
  return OFISTA_OK;
}

ofista_status ofista_echo(ofista_ctx *c, int32_t s, const void *d_rho, const void *d_noise,
                          double snr_db, double phase_err, void *d_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_rho || !d_out || !std::isfinite(snr_db) || !std::isfinite(phase_err)) return OFISTA_E_ARG;
  if (s < 0 || s >= c->L.npos) return OFISTA_E_RANGE;
  OF_CK(c, launch_echo(c->g, c->d.pos, s, static_cast<const float2 *>(d_rho),
                       static_cast<const float2 *>(d_noise), snr_db, phase_err, c->d.echo_tmp,
                       static_cast<float2 *>(d_out), c->st));
  return OFISTA_OK;
}

ofista_status ofista_bp_image(ofista_ctx *c, void *d_img_out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_img_out) return OFISTA_E_ARG;
  if (!c->d.bp || c->n == 0) return OFISTA_E_STATE;
  OF_CK(c, launch_scale(c->d.bp, static_cast<float>(1.0 / static_cast<double>(c->n)), c->L.npix,
                        static_cast<float2 *>(d_img_out), c->st));
  return OFISTA_OK;
}

ofista_status ofista_count_large(ofista_ctx *c, double threshold, int64_t *count) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!count || !std::isfinite(threshold)) return OFISTA_E_ARG;
  OF_CK(c, launch_fill(c->d.counter, 1, 0u, c->st));
  OF_CK(c, launch_count_large(c->d.cbuf[c->G & 1], c->L.N, static_cast<float>(threshold), c->d.counter,
                              c->st));
  unsigned h = 0;
  OF_CK(c, hipMemcpyAsync(&h, c->d.counter, sizeof(unsigned), hipMemcpyDeviceToHost, c->st));
  OF_CK(c, hipStreamSynchronize(c->st));
  *count = static_cast<int64_t>(h);
  return OFISTA_OK;
}

ofista_status ofista_state(ofista_ctx *c, ofista_stats *out) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!out) return OFISTA_E_ARG;
  DevScalars s{};
  const int np = c->L.nparts;
  std::vector<double> sr(2 * np), sm(2 * np);
  const int par = static_cast<int>(c->G & 1);
  OF_CK(c, hipStreamSynchronize(c->st));
  OF_CK(c, hipMemcpy(&s, c->d.scal, sizeof(s), hipMemcpyDeviceToHost));
  if (s.fault) return fail_hip(c, hipErrorLaunchTimeOut, "resident step kernel: a grid barrier timed out");
  OF_CK(c, hipMemcpy(sr.data(), c->d.slots[par], 2 * np * sizeof(double), hipMemcpyDeviceToHost));
  OF_CK(c, hipMemcpy(sm.data(), c->d.slots[par ^ 1], 2 * np * sizeof(double), hipMemcpyDeviceToHost));
  double rho = 0.0;
  if (c->have_iter) {
    double rs = 0.0, ms = 0.0;
    for (int j = 0; j < np; ++j) {
      rs += sr[j];
      ms += sm[np + j];
    }
    rho = rs / ms;
  }
  out->n_pulses = c->n;
  out->n_iters = c->G;
  out->t = c->t;
  out->L = s.L;
  out->tau = s.tau;
  out->lambda = s.lam;
  out->rho = rho;
  out->sigma2 = s.sigma2;
  return OFISTA_OK;
}

}  // extern "C"

namespace {

ofista_status export_to(ofista_ctx *c, void *d_buf) {
  const Layout &L = c->L;
  const int par = static_cast<int>(c->G & 1);
  double hdr[16] = {0};
  hdr[0] = static_cast<double>(c->n);
  hdr[1] = static_cast<double>(c->G);
  hdr[2] = c->t;
  hdr[3] = c->have_iter ? 1.0 : 0.0;
  hdr[6] = c->step_since_push ? 1.0 : 0.0;
  hdr[4] = static_cast<double>(L.N);
  hdr[5] = static_cast<double>(L.K);
  char *o = static_cast<char *>(d_buf);
  const size_t vec = static_cast<size_t>(L.Npad) * sizeof(float2);
  OF_CK(c, hipMemcpyAsync(o, hdr, sizeof(hdr), hipMemcpyHostToDevice, c->st));
  o += align_up(sizeof(hdr));
  OF_CK(c, hipMemcpyAsync(o, c->d.scal, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->st));
  o += align_up(sizeof(DevScalars));
  OF_CK(c, hipMemcpyAsync(o, c->d.slots[par], 2 * L.nparts * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  o += align_up(2 * L.nparts * sizeof(double));
  OF_CK(c, hipMemcpyAsync(o, c->d.slots[par ^ 1], 2 * L.nparts * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  o += align_up(2 * L.nparts * sizeof(double));
  OF_CK(c, hipMemcpyAsync(o, c->d.wbuf[par], vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(o, c->d.cbuf[par], vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(o, c->d.b, vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(o, c->d.H, L.ntiles * kTile * kTile * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
  o += align_up(L.ntiles * kTile * kTile * sizeof(float2));
  if (c->d.bp)
    OF_CK(c, hipMemcpyAsync(o, c->d.bp, static_cast<size_t>(L.npix) * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
  OF_CK(c, hipStreamSynchronize(c->st));  // the header came from host stack memory
  return OFISTA_OK;
}

ofista_status import_from(ofista_ctx *c, const void *d_buf) {
  const Layout &L = c->L;
  double hdr[16];
  const char *o = static_cast<const char *>(d_buf);
  OF_CK(c, hipStreamSynchronize(c->st));
  OF_CK(c, hipMemcpy(hdr, o, sizeof(hdr), hipMemcpyDeviceToHost));
  if (hdr[4] != static_cast<double>(L.N) || hdr[5] != static_cast<double>(L.K)) return OFISTA_E_ARG;
  c->n = static_cast<int64_t>(hdr[0]);
  c->G = static_cast<int64_t>(hdr[1]);
  c->t = hdr[2];
  c->have_iter = hdr[3] != 0.0;
  c->step_since_push = hdr[6] != 0.0;
  const int par = static_cast<int>(c->G & 1);
  const size_t vec = static_cast<size_t>(L.Npad) * sizeof(float2);
  o += align_up(sizeof(hdr));
  OF_CK(c, hipMemcpyAsync(c->d.scal, o, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->st));
  o += align_up(sizeof(DevScalars));
  OF_CK(c, hipMemcpyAsync(c->d.slots[par], o, 2 * L.nparts * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  o += align_up(2 * L.nparts * sizeof(double));
  OF_CK(c, hipMemcpyAsync(c->d.slots[par ^ 1], o, 2 * L.nparts * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  o += align_up(2 * L.nparts * sizeof(double));
  OF_CK(c, hipMemcpyAsync(c->d.wbuf[par], o, vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(c->d.cbuf[par], o, vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(c->d.b, o, vec, hipMemcpyDeviceToDevice, c->st));
  o += align_up(vec);
  OF_CK(c, hipMemcpyAsync(c->d.H, o, L.ntiles * kTile * kTile * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
  o += align_up(L.ntiles * kTile * kTile * sizeof(float2));
  if (c->d.bp)
    OF_CK(c, hipMemcpyAsync(c->d.bp, o, static_cast<size_t>(L.npix) * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
  return OFISTA_OK;
}

}  // namespace

extern "C" {

ofista_status ofista_export_state(ofista_ctx *c, void *d_buf) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_buf) return OFISTA_E_ARG;
  if (c->L.store) return OFISTA_E_UNSUPPORTED;
  return export_to(c, d_buf);
}

ofista_status ofista_import_state(ofista_ctx *c, const void *d_buf) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!d_buf) return OFISTA_E_ARG;
  if (c->L.store) return OFISTA_E_UNSUPPORTED;
  c->rec.clear();  // an imported state has no recorded history
  return import_from(c, d_buf);
}

ofista_status ofista_profile(ofista_ctx *c, int32_t enable) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  OF_CK(c, hipStreamSynchronize(c->st));
  for (auto &p : c->ev) {
    c->pool.push_back(p.second.first);
    c->pool.push_back(p.second.second);
  }
  c->ev.clear();
  c->prof = enable != 0;
  return OFISTA_OK;
}

ofista_status ofista_kernel_time(ofista_ctx *c, int32_t kernel, double *total_ms, int64_t *launches) {
  ofista_status st = usable(c);
  if (st != OFISTA_OK) return st;
  if (!total_ms || !launches || kernel < 0 || kernel >= kProfN) return OFISTA_E_ARG;
  OF_CK(c, hipStreamSynchronize(c->st));
  double tot = 0.0;
  int64_t n = 0;
  for (auto &p : c->ev) {
    if (p.first != kernel) continue;
    float ms = 0.f;
    OF_CK(c, hipEventElapsedTime(&ms, p.second.first, p.second.second));
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return OFISTA_OK;
}

void ofista_destroy(ofista_ctx *c) {
  if (!c) return;
  for (auto &p : c->ev) {
    hipEventDestroy(p.second.first);
    hipEventDestroy(p.second.second);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  delete c;
}

const char *ofista_error_string(const ofista_ctx *c, ofista_status st) {
  if (c && !c->msg.empty() && st == OFISTA_E_HIP) return c->msg.c_str();
  if (c && c->note && st == c->note_st) return c->note;
  return status_text(st);
}

}  // extern "C"
