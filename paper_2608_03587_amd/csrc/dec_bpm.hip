// Host runtime and C ABI of the DEC beam-propagation library (MI355X, gfx950).
//
// A handle owns one "engine": the operators of one mesh (or of a batch of
// meshes concatenated block-diagonally) in device order, the work vectors of
// the z march, and a cache of instantiated hipGraphs of the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/dec_bpm.h"
#include "assembly.hpp"
#include "kernels.hpp"

namespace decbpm {

thread_local std::string g_last_error;

#define HIP_OK(expr)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) fail(DEC_BPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Largest dz * rho(H_lin) accepted: the classical RK4 stability region covers
// the imaginary axis up to 2 sqrt(2); keep a margin below it.
constexpr double kStabilityLimit = 2.5;

// Device copy of a tile set.
struct DevTiles {
  int32_t n_tiles = 0, TS = 0, max_slots = 0, max_compute = 0;
  int32_t* hdr = nullptr;
  int64_t* ent = nullptr;
  int32_t* ext = nullptr;
  int32_t* lsl = nullptr;
  uint16_t* lcol = nullptr;
  void* llw = nullptr;
  void* lmw = nullptr;
  void* llwi = nullptr;  // imaginary part of the L weights (PML handles), else null
  uint8_t* dep = nullptr;  // step layout: depth of each owned slot (see HostTiles)
  int64_t entries = 0, slots = 0;
  int32_t ext_stride = 0, lsl_stride = 0, hdr_stride = 8;

  template <typename T>
  TileOps<T> ops() const {
    TileOps<T> t;
    t.ext_stride = ext_stride;
    t.lsl_stride = lsl_stride;
    t.hdr_stride = hdr_stride;
    t.n_tiles = n_tiles;
    t.TS = TS;
    t.max_slots = max_slots;
    t.max_compute = max_compute;
    t.hdr = hdr;
    t.ent_base = ent;
    t.ext = ext;
    t.lsl = lsl;
    t.lcol = lcol;
    t.llw = static_cast<const T*>(llw);
    t.lmw = static_cast<const T*>(lmw);
    t.llwi = static_cast<const T*>(llwi);
    t.dep = dep;
    return t;
  }
};

struct GraphEntry {
  double dz, gamma;
  int spg, block, xcd, fused, tile_block;  // fused < 0: -(trials) of an adaptive chunk
  hipGraphExec_t exec;
  hipGraph_t graph;
  double rtol = 0.0, atol = 0.0;
};

struct Engine {
  int dtype = DEC_BPM_C64;
  int64_t n_rows = 0;  // device rows
  int32_t F = 1;
  // batches: fields of each mesh in the caller's layout (the device carries F,
  // at least the largest, per row), and per device row its first caller
  // element and its mesh's field count
  std::vector<int32_t> fpm;
  int64_t* bcbase = nullptr;
  int32_t* bfcount = nullptr;
  double p1 = 0.5, beta4 = 0.0;
  double p3 = 0.0, p4 = 0.0;  // coefficients of L^3, L^4
  int nk = DEC_BPM_N_KERR;    // Kerr response
  double npar = 0.0;
  int nl = DEC_BPM_NL_DEC;
  double rho = 0.0;
  double dn_max = 0.0;
  int64_t nnz_off = 0;     // stored off-diagonal neighbours (no padding)
  int64_t n_entries = 0;   // sliced-ELL entries including padding
  bool on_device = false;
  // device operators
  int64_t* sl_info = nullptr;
  int32_t wmax = 0;
  int32_t* col = nullptr;
  void* lw = nullptr;
  void* mw = nullptr;
  void* mdiag = nullptr;
  void* sig = nullptr;  // PML: sigma_p = H0~_p / H0_p (complex, device order), else null
  void* v = nullptr;
  void* v0 = nullptr;
  void* w = nullptr;
  double* h0 = nullptr;
  double* h0c = nullptr;  // caller order
  int32_t* perm = nullptr;
  // tiles of the fused path (F = 1, beta4 = 0) and of the batched path (F > 1)
  bool has_tiles = false;
  bool has_btiles = false;
  int fused = -1;     // launch mode (-1: chosen after the tiles are built)
  int tile_size = 512;
  int tile_block = 256;
  DevTiles tl, bt, stp;  // two-kernel tiles (3 rings), batched tiles, one-kernel-step tiles (5 rings)
  // batches: one-field step tiles over every mesh's rows, for the field-loop
  // step (launch mode 6: a workgroup per tile steps all fields in turn)
  DevTiles sfl;
  bool has_sfl = false;
  // L^3 or L^4: tiles of D halo rings (D = 4 with p4, else 3) for the RK4
  // stages of the operator sum (one tile kernel per stage)
  DevTiles gtl;
  bool has_gtl = false;
  bool gen_tiles = true;  // DEC_BPM_GEN_TILES=0: the gather-kernel chain instead
  int gblock() const {
    const int mc = gtl.max_compute;
    const int b = std::max(tile_block, ((mc + 1) / 2 + 63) / 64 * 64);
    if (b >= mc) return std::min(1024, b);
    return std::min(dtype == DEC_BPM_C128 ? 640 : 1024, b);
  }
  bool has_step = false;
  bool has_step4 = false;  // the step tiles hold the beta4 layout (eight or nine rings)
  bool pml = false;        // complex-stretched L (perfectly matched layer): step-tile kernels only
  int step_tile = 1024;  // rows per tile of the one-kernel step (largest that fits)
  bool sort_ring0 = true;  // step tiles: order the owned rows by degree too
  // persistent stepping on the step tiles: neighbour-tile lists, flags, wait bound
  bool has_persist = false;
  int32_t* nb_ptr = nullptr;
  int32_t* nb_list = nullptr;
  int32_t* pflags = nullptr;
  // flag values of the next persistent launch start above pepoch (flags only
  // grow); INT32_MAX: the flags hold values of another kind and are cleared first
  int32_t pepoch = INT32_MAX;
  // complex128: the step tiles are cut for the one-kernel step's 100 KiB of LDS
  // (512 owned rows), too many to be resident at once; the persistent kernel
  // then gets tiles of its own (1024 owned rows, up to 150 KiB of LDS)
  DevTiles pst;
  bool pst_own = false;
  int spin_limit = 1 << 20;
  // persistent step launches: cooperative (the runtime guarantees residency,
  // about 12 us more per launch) or ordinary (ordered across streams, below)
  bool coop = false;
  int persist_cap_block = -1, persist_cap = 0;  // resident workgroups at that block size
  int persist_cap_block_u = -1, persist_cap_u = 0;  // the same for the unsplit RK4 body
  int mode_cap_block = -1, mode_cap = 0;            // and for the persistent mode iteration
  void* psi2 = nullptr;
  // adaptive Dormand-Prince runs: seven-ring tiles built at the first call from
  // the device-order adjacency kept on the host, the controller state and the
  // per-tile error partials
  struct {
    std::vector<int64_t> arp;
    std::vector<int32_t> col;
    std::vector<double> lw, mw;
    std::vector<double> lwi;  // imaginary parts of the L weights (a PML), else empty
    bool dec = false;
  } adj;
  bool dp5_tried = false, has_dp5 = false;
  int dp5_tile = 1024;        // largest rows per tile tried
  bool dp5_one_slot = false;  // one compute slot per thread (smaller tiles)
  DevTiles dp5;
  Dp5Ctl* dp5ctl = nullptr;
  double* dp5part = nullptr;
  uint32_t* dp5arr = nullptr;
  int32_t* dp5flags = nullptr;
  int dp5_cap_block = -1, dp5_cap = 0;  // resident workgroups of the persistent adaptive kernel
  // nonlinear mode iteration on the step tiles
  ModeCtl* modectl = nullptr;
  double* modepart = nullptr;
  uint32_t* modearr = nullptr;
  // work
  void* psi = nullptr;
  void* ya = nullptr;
  void* yb = nullptr;
  void* t = nullptr;
  void* u = nullptr;  // second Horner buffer of the L^3, L^4 terms
  void* s = nullptr;
  double* partials = nullptr;
  double* red_out = nullptr;
  int* flag = nullptr;
  int n_red_blocks = 1;
  // launch shape
  int block = 256;
  int spg = 32;
  int xcd = 1;
  hipStream_t cap = nullptr;
  std::vector<GraphEntry> graphs;
  std::vector<void*> allocs;
  // records of the recent checkpointed forwards, one per workspace (validated
  // by the adjoint; the oldest is dropped beyond kMaxCkpt)
  struct CkptRec {
    const void* ws = nullptr;
    double dz = 0, gamma = 0;
    int64_t n = -1, every = 0;
    uint64_t dn_digest = 0;
    bool last_recorded = false;  // the workspace holds the last segment's stage vectors
  };
  static constexpr size_t kMaxCkpt = 64;
  std::vector<CkptRec> ckpts;
  // digest of the installed index perturbation's values (0: none), so that
  // installing the same values again restores the same operator identity
  uint64_t dn_digest = 0;

  // threads per workgroup of the step-tile kernels: the requested count if it
  // covers every compute slot once (one slot per thread), else at least half of
  // them (two slots per thread) and at most the two-slot kernels' bound (640
  // threads in complex128, 1024 in complex64)
  int sblock() const {
    const int mc = stp.max_compute;
    const int b = std::max(tile_block, ((mc + 1) / 2 + 63) / 64 * 64);
    if (b >= mc) return std::min(1024, b);
    return std::min(dtype == DEC_BPM_C128 ? 640 : 1024, b);
  }

  // threads per workgroup of the field-loop step (as sblock, on its tiles)
  int fblock() const {
    const int mc = sfl.max_compute;
    const int b = std::max(tile_block, ((mc + 1) / 2 + 63) / 64 * 64);
    if (b >= mc) return std::min(1024, b);
    return std::min(dtype == DEC_BPM_C128 ? 640 : 1024, b);
  }
  // the field-loop kernel stages at most three state slots per thread
  bool use_sfl() const { return has_sfl && F > 1 && sfl.max_slots <= 3 * fblock(); }

  const DevTiles& ptiles() const { return pst_own ? pst : stp; }
  // threads per workgroup of the persistent kernel: as the step kernels on the
  // step tiles; on its own tiles at most two slots per thread of 1024
  int pblock() const {
    if (!pst_own) return sblock();
    const int mc = pst.max_compute;
    return std::min(1024, std::max(tile_block, ((mc + 1) / 2 + 63) / 64 * 64));
  }

  // threads per tile workgroup: the requested count, raised so that no thread
  // owns more than two compute slots of a tile (the fused kernels' register budget)
  int tblock() const {
    const int need = ((tl.max_compute + 1) / 2 + 63) / 64 * 64;
    return std::min(1024, std::max(tile_block, need));
  }

  // L^3, L^4 or a non-Kerr response: the entry points written for the Kerr
  // right-hand side and terms up to L^2 refuse these handles
  bool general() const { return p3 != 0.0 || p4 != 0.0 || nk != DEC_BPM_N_KERR; }
  // terms beyond L^2: the tile kernels' halos cover at most two products per
  // stage, so these run the five-kernel path; a non-Kerr response alone does
  // not (the tile kernels' Kerr phase takes the response's flow integral)
  bool high_order() const { return p3 != 0.0 || p4 != 0.0; }

  size_t real_size() const { return dtype == DEC_BPM_C64 ? 4 : 8; }
  size_t cplx_size() const { return 2 * real_size(); }

  template <typename T>
  TileOps<T> tiles() const {
    return tl.template ops<T>();
  }

  template <typename T>
  DevOps<T> ops() const {
    DevOps<T> d;
    d.n_rows = n_rows;
    d.F = F;
    d.lgF = -1;
    for (int k = 0; k < 31; ++k)
      if ((int64_t(1) << k) == int64_t(F)) d.lgF = k;
    d.wmax = wmax;
    d.sl_info = sl_info;
    d.col = col;
    d.lw = static_cast<const T*>(lw);
    d.mw = static_cast<const T*>(mw);
    d.mdiag = static_cast<const T*>(mdiag);
    d.v = static_cast<const T*>(v);
    d.w = static_cast<const T*>(w);
    d.h0 = h0;
    d.p1 = T(p1);
    d.beta4 = T(beta4);
    d.xcd_remap = xcd;
    d.nk = nk;
    d.npar = T(npar);
    return d;
  }

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(DEC_BPM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    allocs.push_back(p);
    return p;
  }

  void release() {
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }

  void drop_graphs() {
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
  }
};

// Default launch shape from the environment (used before any autotuning).
static void env_defaults(Engine& E) {
  if (const char* s = std::getenv("DEC_BPM_TILE")) E.tile_size = std::max(64, std::min(4096, std::atoi(s)));
  if (const char* s = std::getenv("DEC_BPM_STEP_TILE")) E.step_tile = std::max(64, std::min(4096, std::atoi(s)));
  if (const char* s = std::getenv("DEC_BPM_SPIN_LIMIT")) E.spin_limit = std::max(0, std::atoi(s));
  if (const char* s = std::getenv("DEC_BPM_SORT_RING0")) E.sort_ring0 = std::atoi(s) != 0;
  if (const char* s = std::getenv("DEC_BPM_DP5_TILE")) E.dp5_tile = std::max(64, std::min(1024, std::atoi(s)));
  if (const char* s = std::getenv("DEC_BPM_DP5_ONE_SLOT")) E.dp5_one_slot = std::atoi(s) != 0;
  if (const char* s = std::getenv("DEC_BPM_FUSED")) E.fused = std::max(0, std::min(3, std::atoi(s)));
  if (const char* s = std::getenv("DEC_BPM_BLOCK")) E.block = std::max(64, std::min(1024, std::atoi(s)));
  if (const char* s = std::getenv("DEC_BPM_STEPS_PER_GRAPH")) E.spg = std::max(1, std::atoi(s));
  if (const char* s = std::getenv("DEC_BPM_XCD_REMAP")) E.xcd = std::atoi(s) ? 1 : 0;
  if (const char* s = std::getenv("DEC_BPM_COOPERATIVE")) E.coop = std::atoi(s) != 0;
  if (const char* s = std::getenv("DEC_BPM_GEN_TILES")) E.gen_tiles = std::atoi(s) != 0;
}

template <typename T>
static void upload(Engine& E, void*& dst, const std::vector<T>& src) {
  dst = E.dalloc(src.size() * sizeof(T));
  HIP_OK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Tiles: contiguous ranges of TS device rows plus `rings` halo rings found by
// breadth-first search on the adjacency; the operator rows of rings
// 0..ell_rings-1 are stored again with slot-local 16-bit columns, sliced by
// 64 slots.
struct HostTiles {
  int64_t nt = 0;
  int TS = 0;
  std::vector<int32_t> hdr, ext, lsl;
  std::vector<int64_t> ebase;
  std::vector<uint16_t> lcol;
  // step layout: per slot, the graph distance of an owned row to the nearest
  // row the tile does not own (capped at 7; 0 for halo slots), at the ext stride
  std::vector<uint8_t> dep;
  std::vector<double> llw, lmw, llwi;
  int32_t max_slots = 0, max_compute = 0;
  int32_t ext_stride = 0, lsl_stride = 0;  // step layout: fixed per-tile strides
  int32_t hdr_stride = 8;
};

// Tiles of TS consecutive rows with `rings` halo rings (breadth-first over the
// mesh graph) and the operator rows of the slots in rings 0..ell_rings-1 in
// tile-local sliced ELL (16-bit slot columns).
// Classic layout: ring 0 slot i is row t*TS + i, the halo rows of all tiles
// are concatenated (header holds the offsets), rings sorted by row.
// Step layout: every ring, ring 0 included, is sorted by decreasing degree
// (then row) so the 64-slot slices have nearly uniform width; the halo list
// holds every slot and it and the slice table sit at fixed per-tile strides,
// so a tile finds them without reading its header first.
static bool make_tiles(int64_t n, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                       const std::vector<double>& alw, const std::vector<double>& amw, int TS, int rings,
                       int ell_rings, HostTiles& H, bool step_layout = false, bool sort_ring0 = true,
                       const std::vector<double>* alwi = nullptr) {
  if (rings > (step_layout ? 9 : 5) || ell_rings > rings + 1) fail(DEC_BPM_EINVAL, "internal: unsupported ring count");
  H = HostTiles();
  H.TS = TS;
  H.nt = (n + TS - 1) / TS;
  H.hdr_stride = step_layout ? 16 : 8;
  H.hdr.assign(H.nt * H.hdr_stride, 0);
  H.ebase.resize(H.nt);
  std::vector<int32_t> slot_of(n, -1);
  std::vector<int32_t> slots, ring;
  std::vector<std::vector<int32_t>> ext_t, lsl_t;
  std::vector<std::vector<uint8_t>> dep_t;
  if (step_layout) {
    ext_t.resize(H.nt);
    lsl_t.resize(H.nt);
  }
  auto deg = [&](int32_t r) { return arp[r + 1] - arp[r]; };
  for (int64_t t = 0; t < H.nt; ++t) {
    const int64_t r0 = t * TS, r1 = std::min(n, r0 + TS);
    slots.clear();
    for (int64_t r = r0; r < r1; ++r) {
      slot_of[r] = int32_t(r - r0);
      slots.push_back(int32_t(r));
    }
    int cnt[10] = {int(r1 - r0), 0, 0, 0, 0, 0, 0, 0, 0, 0};
    size_t start = 0, end = slots.size();
    for (int k = 1; k <= rings; ++k) {
      ring.clear();
      for (size_t i = start; i < end; ++i)
        for (int64_t e = arp[slots[i]]; e < arp[slots[i] + 1]; ++e)
          if (slot_of[acol[e]] == -1) {
            slot_of[acol[e]] = -2;
            ring.push_back(acol[e]);
          }
      std::sort(ring.begin(), ring.end());
      for (int32_t q : ring) {
        slot_of[q] = int32_t(slots.size());
        slots.push_back(q);
      }
      cnt[k] = int(ring.size());
      start = end;
      end = slots.size();
    }
    if (slots.size() >= 65535) {
      for (int32_t r : slots) slot_of[r] = -1;
      return false;
    }
    if (step_layout) {
      size_t b = 0;
      for (int k = 0; k <= rings; ++k) {
        if (k > 0 || sort_ring0)
          std::stable_sort(slots.begin() + b, slots.begin() + b + cnt[k],
                           [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
        b += cnt[k];
      }
      for (size_t i = 0; i < slots.size(); ++i) slot_of[slots[i]] = int32_t(i);
    }
    if (step_layout) {  // depth of each owned slot: breadth-first from the ring-1 rows inwards
      std::vector<uint8_t> dd(slots.size(), 0);
      std::vector<int32_t> frontier, next;
      const int n0 = cnt[0];
      for (int i = n0; i < n0 + cnt[1]; ++i) frontier.push_back(slots[i]);
      std::vector<uint8_t> seen(slots.size(), 0);
      for (int i = n0; i < int(slots.size()); ++i) seen[i] = 1;
      for (uint8_t dist = 1; dist <= 7 && !frontier.empty(); ++dist) {
        next.clear();
        for (int32_t r : frontier)
          for (int64_t e = arp[r]; e < arp[r + 1]; ++e) {
            const int32_t q = slot_of[acol[e]];
            if (q >= 0 && q < n0 && !seen[q]) {
              seen[q] = 1;
              dd[q] = dist;
              next.push_back(acol[e]);
            }
          }
        frontier.swap(next);
      }
      for (int i = 0; i < n0; ++i)
        if (!seen[i]) dd[i] = 7;  // farther than 7 (or a tile without halo)
      dep_t.push_back(std::move(dd));
    }
    int32_t* h = &H.hdr[t * H.hdr_stride];
    if (step_layout) {  // cumulative counts of rings 0..k, ring count (offsets come from the strides)
      int c = 0;
      for (int k = 0; k < 10; ++k) h[k] = (c += cnt[k]);
      h[15] = rings;
      ext_t[t] = slots;
    } else if (rings <= 3) {  // counts of rings 0..3, ext base, slice-table base
      for (int k = 0; k < 4; ++k) h[k] = cnt[k];
      h[4] = int32_t(H.ext.size());
      h[5] = int32_t(H.lsl.size());
      H.ext.insert(H.ext.end(), slots.begin() + cnt[0], slots.end());
    } else {  // counts of rings 0..5, ext base, slice-table base
      for (int k = 0; k < 6; ++k) h[k] = cnt[k];
      h[6] = int32_t(H.ext.size());
      h[7] = int32_t(H.lsl.size());
      H.ext.insert(H.ext.end(), slots.begin() + cnt[0], slots.end());
    }
    int ce = 0;
    for (int k = 0; k < ell_rings; ++k) ce += cnt[k];
    H.max_compute = std::max(H.max_compute, ce);
    H.ebase[t] = int64_t(H.lcol.size());
    for (int sl = 0; sl * 64 < ce; ++sl) {
      int W = 0;
      for (int i = sl * 64; i < std::min(ce, sl * 64 + 64); ++i) W = std::max<int>(W, int(deg(slots[i])));
      const int64_t rel = int64_t(H.lcol.size()) - H.ebase[t];
      (step_layout ? lsl_t[t] : H.lsl).push_back(int32_t((rel << 8) | W));
      const size_t b = H.lcol.size();
      H.lcol.resize(b + size_t(W) * 64, 0);
      H.llw.resize(b + size_t(W) * 64, 0.0);
      H.lmw.resize(b + size_t(W) * 64, 0.0);
      if (alwi) H.llwi.resize(b + size_t(W) * 64, 0.0);
      for (int lane = 0; lane < 64; ++lane) {
        const int i = sl * 64 + lane;
        for (int k = 0; k < W; ++k) H.lcol[b + size_t(k) * 64 + lane] = uint16_t(i < ce ? i : 0);  // padding: self
        if (i >= ce) continue;
        int k = 0;
        for (int64_t e = arp[slots[i]]; e < arp[slots[i] + 1]; ++e, ++k) {
          const int32_t q = slot_of[acol[e]];
          if (q < 0) fail(DEC_BPM_EINVAL, "internal: halo ring incomplete");
          H.lcol[b + size_t(k) * 64 + lane] = uint16_t(q);
          H.llw[b + size_t(k) * 64 + lane] = alw[e];
          H.lmw[b + size_t(k) * 64 + lane] = amw[e];
          if (alwi) H.llwi[b + size_t(k) * 64 + lane] = (*alwi)[e];
        }
      }
    }
    if (int64_t(H.lcol.size()) - H.ebase[t] >= (int64_t(1) << 23)) fail(DEC_BPM_EINVAL, "tile operator too large");
    H.max_slots = std::max<int32_t>(H.max_slots, int32_t(slots.size()));
    for (int32_t r : slots) slot_of[r] = -1;
  }
  H.max_slots = (H.max_slots + 3) / 4 * 4;
  if (step_layout) {
    for (int64_t t = 0; t < H.nt; ++t) {
      H.ext_stride = std::max<int32_t>(H.ext_stride, int32_t(ext_t[t].size()));
      H.lsl_stride = std::max<int32_t>(H.lsl_stride, int32_t(lsl_t[t].size()));
    }
    H.ext_stride = (H.ext_stride + 63) / 64 * 64;
    H.lsl_stride = std::max<int32_t>(1, (H.lsl_stride + 15) / 16 * 16);
    H.ext.assign(size_t(H.nt) * H.ext_stride, 0);
    H.lsl.assign(size_t(H.nt) * H.lsl_stride, 0);
    H.dep.assign(size_t(H.nt) * H.ext_stride, 0);
    for (int64_t t = 0; t < H.nt; ++t) {
      std::copy(ext_t[t].begin(), ext_t[t].end(), H.ext.begin() + t * H.ext_stride);
      std::copy(lsl_t[t].begin(), lsl_t[t].end(), H.lsl.begin() + t * H.lsl_stride);
      std::copy(dep_t[t].begin(), dep_t[t].end(), H.dep.begin() + t * H.ext_stride);
    }
  }
  if (H.ext.empty()) H.ext.push_back(0);
  if (H.lsl.empty()) H.lsl.push_back(0);
  return true;
}

template <typename T>
static void upload_tiles(Engine& E, const HostTiles& H, bool dec, int64_t n, DevTiles& D) {
  void* p;
  upload(E, p, H.hdr);
  D.hdr = static_cast<int32_t*>(p);
  upload(E, p, H.ebase);
  D.ent = static_cast<int64_t*>(p);
  upload(E, p, H.ext);
  D.ext = static_cast<int32_t*>(p);
  upload(E, p, H.lsl);
  D.lsl = static_cast<int32_t*>(p);
  upload(E, p, H.lcol);
  D.lcol = static_cast<uint16_t*>(p);
  if (!H.dep.empty()) {
    upload(E, p, H.dep);
    D.dep = static_cast<uint8_t*>(p);
  }
  std::vector<T> w(H.llw.begin(), H.llw.end());
  upload(E, D.llw, w);
  if (!H.llwi.empty()) {
    std::vector<T> wi(H.llwi.begin(), H.llwi.end());
    upload(E, D.llwi, wi);
  }
  if (dec) {
    std::vector<T> m(H.lmw.begin(), H.lmw.end());
    upload(E, D.lmw, m);
  }
  D.n_tiles = int32_t(H.nt);
  D.TS = H.TS;
  D.max_slots = H.max_slots;
  D.max_compute = H.max_compute;
  D.entries = int64_t(H.lcol.size());
  D.slots = int64_t(H.ext.size()) + n;
  D.ext_stride = H.ext_stride;
  D.lsl_stride = H.lsl_stride;
  D.hdr_stride = H.hdr_stride;
}

// Plain fused path: the largest tile size (from the requested one, halving)
// whose biggest tile with three halo rings fits 64 KB of LDS and whose
// compute slots fit two per thread of a 1024-thread workgroup.
template <typename T>
static void build_tiles(Engine& E, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                        const std::vector<double>& alw, const std::vector<double>& amw, bool dec) {
  // the tile kernels unroll the neighbour loop to at most 12 entries; wider
  // rows (degree 13 and 14 pass the 25-degree angle bound) take the row kernels
  if (E.wmax > 12) return;
  HostTiles H;
  for (int ts = E.tile_size; ts >= 64; ts /= 2) {
    if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, 3, 3, H)) continue;
    if (size_t(H.max_slots) * 7 * sizeof(T) > 64 * 1024 || H.max_compute > 2 * 1024) continue;
    upload_tiles<T>(E, H, dec, E.n_rows, E.tl);
    E.tile_size = ts;
    E.has_tiles = true;
    return;
  }
}

// One-kernel-per-step path: tiles with five halo rings (four for the lumped
// Kerr term) whose state, stage vectors and |psi|^2 phi fit 64 KB of LDS.
template <typename T>
static void build_step_tiles(Engine& E, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                             const std::vector<double>& alw, const std::vector<double>& amw, bool dec,
                             const std::vector<double>* alwi = nullptr) {
  if (E.wmax > 12) return;
  // without beta4: five rings (four for the lumped Kerr term), 7 reals of LDS
  // per slot; with beta4: two rings per stage, nine (eight), 9 reals per slot;
  // batched handles: VF fields per slot (32 bytes of each state vector), no beta4
  const bool b4 = E.beta4 != 0.0;
  const bool batched = E.F > 1;
  const int VF = int(32 / (2 * sizeof(T)));  // fields per slot of the batched step kernel
  if (batched && (b4 || E.F % VF != 0)) return;
  const int rings = (b4 ? 8 : 4) + (dec ? 1 : 0);
  const size_t lds_reals = batched ? size_t(7 * VF) : (b4 ? 9 : 7);
  // LDS per workgroup: 63 KiB in complex64 (two workgroups then share a CU's
  // 160 KiB).  Complex128 may use up to 100 KiB, so that its tiles keep 512
  // owned rows (the halo work of 256-row tiles doubles it).  The complex64
  // beta4 step, one workgroup per CU either way, may use up to 150 KiB, so that
  // its nine-ring tiles can keep 1024 owned rows (less halo work per owned
  // row); it also takes three compute slots per thread.
  const size_t lds_max = batched ? 150 * 1024
                                 : (b4 ? (sizeof(T) == 8 ? 100 : 150) * 1024 : (sizeof(T) == 8 ? 100 * 1024 : 63 * 1024));
  const int max_compute = sizeof(T) == 8 ? 2 * 640 : (b4 ? 3 : 2) * 1024;
  HostTiles H;
  bool built = false;
  for (int ts = E.step_tile; ts >= 64; ts /= 2) {
    if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, rings, rings, H, true, E.sort_ring0, alwi)) continue;
    if (size_t(H.max_slots) * lds_reals * sizeof(T) > lds_max || H.max_compute > max_compute) continue;
    upload_tiles<T>(E, H, dec, E.n_rows, E.stp);
    (b4 ? E.has_step4 : E.has_step) = true;
    E.step_tile = ts;
    built = true;
    break;
  }
  // the persistent kernel: one-field operators without beta4; complex L (a PML) in complex64 only
  if (!built || b4 || batched || (alwi && sizeof(T) == 8)) return;
  if (sizeof(T) == 8) {
    HostTiles H2;
    for (int ts = 1024; ts > E.step_tile; ts /= 2) {  // larger than the step tiles: fewer to keep resident
      if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, rings, rings, H2, true, E.sort_ring0)) continue;
      if (size_t(H2.max_slots) * 7 * sizeof(T) > 150 * 1024 || H2.max_compute > 2048) continue;
      upload_tiles<T>(E, H2, dec, E.n_rows, E.pst);
      E.pst_own = true;
      H = std::move(H2);
      break;
    }
  }
  // tiles owning the halo rows of each tile (the persistent kernel's wait set)
  std::vector<int32_t> ptr(H.nt + 1, 0), list, seen(H.nt, -1);
  bool fits = true;
  for (int64_t t = 0; t < H.nt; ++t) {
    const int32_t* h = &H.hdr[t * H.hdr_stride];
    const int32_t halo = h[h[15]] - h[0];
    int cnt = 0;
    for (int32_t i = 0; i < halo; ++i) {
      const int32_t u = int32_t(H.ext[t * H.ext_stride + h[0] + i] / H.TS);
      if (u == t || seen[u] == int32_t(t)) continue;
      seen[u] = int32_t(t);
      list.push_back(u);
      ++cnt;
    }
    if (cnt > 64) fits = false;
    ptr[t + 1] = int32_t(list.size());
  }
  if (!fits) return;
  if (list.empty()) list.push_back(0);
  void* p;
  upload(E, p, ptr);
  E.nb_ptr = static_cast<int32_t*>(p);
  upload(E, p, list);
  E.nb_list = static_cast<int32_t*>(p);
  E.pflags = static_cast<int32_t*>(E.dalloc(size_t(H.nt) * sizeof(int32_t)));
  E.has_persist = true;
}

// Operator sums with L^3 or L^4: tiles of D halo rings (D = 4 with p4, else
// 3), three complex vectors per slot in LDS (the stage input and two Horner
// intermediates), for one tile kernel per RK4 stage.
template <typename T>
static void build_gen_tiles(Engine& E, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                            const std::vector<double>& alw, const std::vector<double>& amw) {
  if (!E.high_order() || !E.gen_tiles || E.F != 1 || E.wmax > 12) return;
  const int rings = E.p4 != 0.0 ? 4 : 3;
  const size_t lds_max = sizeof(T) == 8 ? 100 * 1024 : 63 * 1024;  // three complex vectors per slot
  const int max_compute = sizeof(T) == 8 ? 2 * 640 : 2 * 1024;
  HostTiles H;
  for (int ts = 1024; ts >= 64; ts /= 2) {
    if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, rings, rings, H, true, E.sort_ring0)) continue;
    if (size_t(H.max_slots) * 6 * sizeof(T) > lds_max || H.max_compute > max_compute) continue;
    upload_tiles<T>(E, H, false, E.n_rows, E.gtl);
    E.has_gtl = true;
    return;
  }
}

// Batched path, field-loop step: the one-field step tiles (five rings, four
// for the lumped Kerr term) over the concatenated rows of every mesh; a tile
// may straddle two meshes (the operator is block diagonal, so its halo holds
// only rows of the meshes it covers).
template <typename T>
static void build_field_tiles(Engine& E, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                              const std::vector<double>& alw, const std::vector<double>& amw, bool dec) {
  if (E.wmax > 12 || E.beta4 != 0.0) return;
  const int rings = 4 + (dec ? 1 : 0);
  const size_t lds_max = sizeof(T) == 8 ? 100 * 1024 : 63 * 1024;
  const int max_compute = sizeof(T) == 8 ? 2 * 640 : 2 * 1024;
  HostTiles H;
  for (int ts = 1024; ts >= 64; ts /= 2) {
    if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, rings, rings, H, true, E.sort_ring0)) continue;
    if (size_t(H.max_slots) * 7 * sizeof(T) > lds_max || H.max_compute > max_compute) continue;
    upload_tiles<T>(E, H, dec, E.n_rows, E.sfl);
    E.has_sfl = true;
    return;
  }
}

// Batched path: tiles of one halo ring whose field values (all F fields of
// every slot) are staged in LDS by one workgroup; rows per tile so that a
// workgroup has at most 1024 threads of 32 bytes of fields each.
template <typename T>
static void build_batch_tiles(Engine& E, const std::vector<int64_t>& arp, const std::vector<int32_t>& acol,
                              const std::vector<double>& alw, const std::vector<double>& amw, bool dec) {
  const int VF = int(32 / (2 * sizeof(T)));
  if (E.F < VF || E.F % VF || E.wmax > 12) return;
  const int tpr = E.F / VF;  // threads per row
  HostTiles H;
  for (int ts = std::max(1, 1024 / tpr); ts >= 8; ts /= 2) {
    if (!make_tiles(E.n_rows, arp, acol, alw, amw, ts, 1, 1, H)) continue;
    if (size_t(H.max_slots) * E.F * 2 * sizeof(T) > 64 * 1024) continue;
    upload_tiles<T>(E, H, dec, E.n_rows, E.bt);
    E.has_btiles = true;
    return;
  }
}

// Build the device engine from one or more assembled meshes (concatenated).
// Ordinary launches of the persistent step are ordered across the process's
// streams: a launch on a stream other than the device's previous one first
// waits for that launch (two partly resident grids could otherwise wait on
// each other until their bounded waits give up).  On one stream the order is
// the stream's own.  The event is created with the handle, so that launching
// allocates nothing.
struct PersistOrder {
  std::mutex mu;
  hipEvent_t ev = nullptr;
  hipStream_t last = nullptr;
  bool has = false;
};
static PersistOrder g_porder[64];

static void persist_order_init() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lock(g_porder[dev].mu);
  if (!g_porder[dev].ev) HIP_OK(hipEventCreateWithFlags(&g_porder[dev].ev, hipEventDisableTiming));
}

template <typename T>
static void build_engine_t(Engine& E, const std::vector<const Assembled*>& meshes, const std::vector<int>& lumped) {
  int64_t n = 0;
  for (auto* a : meshes) n += a->n;
  E.n_rows = n;
  const int64_t n_sl = (n + 63) / 64;
  std::vector<int64_t> sl_off(n_sl + 1, 0);
  std::vector<int32_t> sl_w(n_sl, 0);
  // per device row: mesh id, local row
  std::vector<int32_t> row_mesh(n), row_local(n);
  std::vector<int64_t> mesh_off(meshes.size() + 1, 0);
  for (size_t m = 0; m < meshes.size(); ++m) mesh_off[m + 1] = mesh_off[m] + meshes[m]->n;
  for (size_t m = 0; m < meshes.size(); ++m)
    for (int64_t i = 0; i < meshes[m]->n; ++i) {
      row_mesh[mesh_off[m] + i] = int32_t(m);
      row_local[mesh_off[m] + i] = int32_t(i);
    }
  auto degree = [&](int64_t r) {
    const Assembled& a = *meshes[row_mesh[r]];
    const int32_t p = a.perm[row_local[r]];
    return int32_t(a.rp[p + 1] - a.rp[p] - 1);
  };
  E.nnz_off = 0;
  for (int64_t s = 0; s < n_sl; ++s) {
    int32_t wmax = 0;
    for (int64_t r = s * 64; r < std::min(n, (s + 1) * 64); ++r) {
      int32_t dg = degree(r);
      wmax = std::max(wmax, dg);
      E.nnz_off += dg;
    }
    sl_w[s] = wmax;
    sl_off[s + 1] = sl_off[s] + int64_t(wmax) * 64;
  }
  E.n_entries = sl_off[n_sl];
  std::vector<int32_t> col(E.n_entries, 0);
  std::vector<T> lw(E.n_entries, T(0)), mw(E.n_entries, T(0));
  std::vector<T> mdiag(n), v0(n), w(n);
  std::vector<double> h0(n), h0c(n);
  std::vector<int32_t> perm(n);
  bool any_dec = false;
  // device-order adjacency (kept on the host to build the tiles)
  std::vector<int64_t> arp(n + 1, 0);
  std::vector<int32_t> acol;
  std::vector<double> alw, amw, alwi;
  // a perfectly matched layer makes L complex: c_pq = -K~_pq / H0~_p
  const bool pml = meshes.size() == 1 && !meshes[0]->kp_re.empty();
  E.pml = pml;
  std::vector<T> sig;  // PML: sigma_p = H0~_p / H0_p per row (device order), interleaved complex
  if (pml) sig.resize(size_t(2) * n);
  acol.reserve(E.nnz_off);
  alw.reserve(E.nnz_off);
  amw.reserve(E.nnz_off);
  for (int64_t r = 0; r < n; ++r) {
    const int m = row_mesh[r];
    const Assembled& a = *meshes[m];
    const int64_t off = mesh_off[m];
    const int32_t p = a.perm[row_local[r]];
    const double hp = a.h0[p];
    perm[r] = int32_t(off + p);
    h0[r] = hp;
    h0c[off + p] = hp;
    if (pml) {
      sig[2 * r] = T(a.h0p_re[p] / hp);
      sig[2 * r + 1] = T(a.h0p_im[p] / hp);
    }
    v0[r] = T(a.v[p]);
    w[r] = T(a.w[p]);
    // neighbours sorted by device column
    std::vector<std::pair<int32_t, int64_t>> nb;
    for (int64_t e = a.rp[p]; e < a.rp[p + 1]; ++e) {
      if (a.col[e] == p) {
        mdiag[r] = T(lumped[m] ? a.chibar[p] : a.qdq[e] / hp);
        continue;
      }
      nb.emplace_back(int32_t(off + a.iperm[a.col[e]]), e);
    }
    std::sort(nb.begin(), nb.end());
    for (auto& e : nb) {
      acol.push_back(e.first);
      if (pml) {
        const std::complex<double> c =
            -std::complex<double>(a.kp_re[e.second], a.kp_im[e.second]) / std::complex<double>(a.h0p_re[p], a.h0p_im[p]);
        alw.push_back(c.real());
        alwi.push_back(c.imag());
      } else {
        alw.push_back(-a.k[e.second] / hp);
      }
      amw.push_back(lumped[m] ? 0.0 : a.qdq[e.second] / hp);
    }
    arp[r + 1] = int64_t(acol.size());
    const int64_t s = r >> 6, lane = r & 63;
    for (int k = 0; k < sl_w[s]; ++k) {
      const int64_t slot = sl_off[s] + int64_t(k) * 64 + lane;
      if (k < int(nb.size())) {
        col[slot] = nb[k].first;
        lw[slot] = T(pml ? alw[arp[r] + k] : -a.k[nb[k].second] / hp);  // PML: real part (diagnostics only)
        mw[slot] = lumped[m] ? T(0) : T(a.qdq[nb[k].second] / hp);
      } else {
        col[slot] = int32_t(r);  // padding: self, zero weights
      }
    }
    if (!lumped[m]) any_dec = true;
  }
  // lanes past the last row of the last slice
  for (int64_t r = n; r < n_sl * 64; ++r) {
    const int64_t s = r >> 6, lane = r & 63;
    for (int k = 0; k < sl_w[s]; ++k) col[sl_off[s] + int64_t(k) * 64 + lane] = 0;
  }
  std::vector<int64_t> sl_info(n_sl);
  E.wmax = 0;
  for (int64_t s = 0; s < n_sl; ++s) {
    if (sl_w[s] > 255) fail(DEC_BPM_EMESH, "a vertex has more than 255 neighbours");
    sl_info[s] = (sl_off[s] << 8) | int64_t(sl_w[s]);
    E.wmax = std::max(E.wmax, sl_w[s]);
  }
  void* p;
  upload(E, p, sl_info);
  E.sl_info = static_cast<int64_t*>(p);
  upload(E, p, col);
  E.col = static_cast<int32_t*>(p);
  upload(E, E.lw, lw);
  if (any_dec) upload(E, E.mw, mw);
  upload(E, E.mdiag, mdiag);
  if (pml) upload(E, E.sig, sig);
  upload(E, E.v0, v0);
  upload(E, E.v, v0);
  upload(E, E.w, w);
  upload(E, p, h0);
  E.h0 = static_cast<double*>(p);
  upload(E, p, h0c);
  E.h0c = static_cast<double*>(p);
  upload(E, p, perm);
  E.perm = static_cast<int32_t*>(p);
  if (E.F > 1) {  // caller element of each device row's first field
    std::vector<int64_t> ebase(meshes.size() + 1, 0), cbase(n);
    std::vector<int32_t> fcount(n);
    for (size_t m = 0; m < meshes.size(); ++m) ebase[m + 1] = ebase[m] + meshes[m]->n * E.fpm[m];
    for (int64_t r = 0; r < n; ++r) {
      const int m = row_mesh[r];
      cbase[r] = ebase[m] + (int64_t(perm[r]) - mesh_off[m]) * E.fpm[m];
      fcount[r] = E.fpm[m];
    }
    upload(E, p, cbase);
    E.bcbase = static_cast<int64_t*>(p);
    upload(E, p, fcount);
    E.bfcount = static_cast<int32_t*>(p);
  }
  if (E.F == 1 && E.beta4 == 0.0 && !pml && !E.high_order()) build_tiles<T>(E, arp, acol, alw, amw, any_dec);
  if (!E.high_order()) build_step_tiles<T>(E, arp, acol, alw, amw, any_dec, pml ? &alwi : nullptr);
  if (pml && !E.has_step)
    fail(DEC_BPM_EINVAL, "PML: the mesh needs the one-kernel step tiles (rows of at most 12 neighbours)");
  if (E.F > 1) build_batch_tiles<T>(E, arp, acol, alw, amw, any_dec);
  if (E.F > 1 && !E.general()) build_field_tiles<T>(E, arp, acol, alw, amw, any_dec);
  build_gen_tiles<T>(E, arp, acol, alw, amw);
  if (E.has_step && E.F == 1) {  // kept for the adaptive integrator's tiles
    E.adj.arp = std::move(arp);
    E.adj.col = std::move(acol);
    E.adj.lw = std::move(alw);
    E.adj.mw = std::move(amw);
    if (pml) E.adj.lwi = std::move(alwi);
    E.adj.dec = any_dec;
  }
  const size_t nv = size_t(n) * E.F;
  E.psi = E.dalloc(nv * 2 * sizeof(T));
  if (E.has_tiles || E.has_step || E.has_step4 || E.has_sfl) E.psi2 = E.dalloc(nv * 2 * sizeof(T));
  E.ya = E.dalloc(nv * 2 * sizeof(T));
  E.yb = E.dalloc(nv * 2 * sizeof(T));
  E.t = (E.beta4 != 0.0 || E.general()) ? E.dalloc(nv * 2 * sizeof(T)) : nullptr;
  E.u = (E.p3 != 0.0 || E.p4 != 0.0) ? E.dalloc(nv * 2 * sizeof(T)) : nullptr;
  E.s = E.dalloc(nv * sizeof(T));
  E.n_red_blocks = int((n + 255) / 256);
  E.partials = static_cast<double*>(E.dalloc(2 * size_t(std::max(E.n_red_blocks, 1)) * sizeof(double)));
  E.red_out = static_cast<double*>(E.dalloc(2 * sizeof(double)));
  E.flag = static_cast<int*>(E.dalloc(sizeof(int)));
  HIP_OK(hipMemset(E.flag, 0, sizeof(int)));
  HIP_OK(hipStreamCreateWithFlags(&E.cap, hipStreamNonBlocking));
  persist_order_init();
  E.on_device = true;
}

static void build_engine(Engine& E, const std::vector<const Assembled*>& meshes, const std::vector<int>& lumped) {
  env_defaults(E);
  if (E.dtype == DEC_BPM_C64)
    build_engine_t<float>(E, meshes, lumped);
  else
    build_engine_t<double>(E, meshes, lumped);
  if (E.fused < 0) E.fused = (E.has_step || E.has_step4) ? 2 : ((E.has_tiles || E.has_btiles) ? 1 : 0);
  if (E.pml) E.fused = 2;
  if (E.high_order()) E.fused = 0;
}

static void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(DEC_BPM_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

// ---- one z step on the engine's device-order state psi (F fields per row) ----
// LIN(dz) as a Horner evaluation of the RK4 polynomial (identical to the four
// classical stages for a linear autonomous system), then NL(tau_next).
// Batched engines with tiles run the LDS-tiled kernels (same arithmetic).
template <typename T>
static bool use_btiles(const Engine& E) {
  return E.has_btiles && E.fused;
}

template <typename T>
static void do_stage(const Engine& E, const DevOps<T>& d, const void* x, const void* t, const void* psi, void* y,
                     double coef, void* s_out, double tau_s, hipStream_t st) {
  if (use_btiles<T>(E))
    launch_bstage<T>(d, E.bt.template ops<T>(), x, t, psi, y, coef, s_out, tau_s, st);
  else
    launch_stage<T>(d, x, t, psi, y, coef, s_out, tau_s, E.block, st);
}

template <typename T>
static void do_lap(const Engine& E, const DevOps<T>& d, const void* x, void* t, hipStream_t st) {
  if (use_btiles<T>(E))
    launch_blap<T>(d, E.bt.template ops<T>(), x, t, st);
  else
    launch_lap<T>(d, x, t, E.block, st);
}

// The Kerr step stays row-parallel: its gathered vector (|psi|^2 phi, real)
// is half the size of a field and the tiled variant measured slower.
template <typename T>
static void do_kerr(const Engine& E, const DevOps<T>& d, const void* in, void* out, const void* s, double tau,
                    double gamma, hipStream_t st) {
  launch_kerr<T>(d, in, out, s, tau, gamma, E.block, st);
}

template <typename T>
static void lin_step(const Engine& E, const DevOps<T>& d, const void* in, void* out, void* y1, void* y2, void* y3,
                     double dz, void* s_out, double tau_s, hipStream_t st) {
  const void* t = nullptr;
  // y1 = psi + dz/4 A psi;  y2 = psi + dz/3 A y1;  y3 = psi + dz/2 A y2;  out = psi + dz A y3
  const void* xs[4] = {in, y1, y2, y3};
  void* ys[4] = {y1, y2, y3, out};
  const double cs[4] = {dz / 4, dz / 3, dz / 2, dz};
  if ((E.p3 != 0.0 || E.p4 != 0.0) && E.has_gtl) {
    // one tile kernel per stage: the Horner chain of the operator sum in LDS
    const TileOps<T> tg = E.gtl.template ops<T>();
    for (int k = 0; k < 4; ++k)
      launch_hstage<T>(d, tg, xs[k], in, ys[k], cs[k], E.p3, E.p4, k == 3 ? s_out : nullptr, tau_s, E.gblock(), st);
    return;
  }
  if (E.p3 != 0.0 || E.p4 != 0.0) {
    // sum_n p_n L^n x = L U with U = p1 x + L(p2 x + L(p3 x + p4 L x)) by Horner;
    // the beta4 stage with p1 -> 0, beta4 -> 1 and t = U applies the last L
    DevOps<T> dg = d;
    dg.p1 = T(0);
    dg.beta4 = T(1);
    for (int k = 0; k < 4; ++k) {
      const void* x = xs[k];
      if (E.p4 != 0.0) {
        launch_lapc<T>(d, x, x, E.p4, E.p3, E.t, E.block, st);    // p3 x + p4 L x
        launch_lapc<T>(d, E.t, x, 1.0, E.beta4, E.u, E.block, st);  // p2 x + L(.)
      } else {
        launch_lapc<T>(d, x, x, E.p3, E.beta4, E.u, E.block, st);   // p2 x + p3 L x
      }
      launch_lapc<T>(d, E.u, x, 1.0, E.p1, E.t, E.block, st);      // U = p1 x + L(.)
      do_stage<T>(E, dg, x, E.t, in, ys[k], cs[k], k == 3 ? s_out : nullptr, tau_s, st);
    }
    return;
  }
  for (int k = 0; k < 4; ++k) {
    if (E.beta4 != 0.0) {
      do_lap<T>(E, d, xs[k], E.t, st);
      t = E.t;
    }
    do_stage<T>(E, d, xs[k], t, in, ys[k], cs[k], k == 3 ? s_out : nullptr, tau_s, st);
  }
}

template <typename T>
static void z_step(const Engine& E, const DevOps<T>& d, double dz, double gamma, double tau_next, hipStream_t st) {
  // buffers: y1 -> ya, y2 -> yb, y3 -> ya (y1 is dead once y2 exists), result in place on psi
  lin_step<T>(E, d, E.psi, E.psi, E.ya, E.yb, E.ya, dz, E.s, tau_next, st);
  do_kerr<T>(E, d, E.psi, E.psi, E.s, tau_next, gamma, st);
}

// fused: 0 = five kernels per step, 1 = two tile kernels per step, 2 = one tile kernel per step
template <typename T>
static bool use_fused(const Engine& E) {
  return E.has_tiles && E.fused == 1;
}

template <typename T>
static bool use_step(const Engine& E) {
  return E.has_step && E.fused == 2;
}

// Checkpointed forward and adjoint on the step tiles (launch modes 2 and 3).
template <typename T>
static bool use_step_adjoint(const Engine& E) {
  return E.has_step && E.fused >= 2 && size_t(E.stp.max_slots) * 3 * 2 * sizeof(T) <= 64 * 1024;
}

// Persistent stepping needs every step tile resident at once (body 0: the
// split step, 1: the unsplit RK4 step).
template <typename T>
static bool persist_fits(Engine& E, int body = 0) {
  if (!E.has_persist) return false;
  const int b = E.pblock();
  int& cap_block = body ? E.persist_cap_block_u : E.persist_cap_block;
  int& cap = body ? E.persist_cap_u : E.persist_cap;
  if (cap_block != b) {
    cap = persist_capacity<T>(E.ops<T>(), E.ptiles().template ops<T>(), b, body);
    cap_block = b;
  }
  const int64_t grid = E.xcd ? (int64_t(E.ptiles().n_tiles) + 7) / 8 * 8 : E.ptiles().n_tiles;  // as launched
  return cap >= grid;
}

template <typename T>
static bool use_persist(Engine& E) {
  return E.fused == 3 && persist_fits<T>(E);
}

// One fused middle z step: state cur (psi after NL) and y1 in ya -> next state in nxt, its y1 in ya.
template <typename T>
static void fused_mid(const Engine& E, const DevOps<T>& d, const TileOps<T>& tl, void* cur, void* nxt, double dz,
                      double gamma, hipStream_t st) {
  launch_fused<T>(d, tl, FUSED_S2_S3, E.ya, cur, nullptr, E.yb, nullptr, dz, dz, gamma, E.tblock(), st);
  launch_fused<T>(d, tl, FUSED_S4_NL_S1, E.yb, cur, nxt, E.ya, nullptr, dz, dz, gamma, E.tblock(), st);
}

// Launch mode of the middle steps: 0 = five kernels (nine with beta4), 1 = two
// tile kernels, 2 = one tile kernel per step, 3 = one persistent launch for all
// of them, 4 = one tile kernel per step with the beta4 term (modes whose tiles
// are missing fall back to the row kernels).  Mode 5, one unsplit RK4 step per
// tile kernel, is only requested explicitly (dec_bpm_propagate_unsplit).
// Mode 6 (batches, fused = 3): one field-loop tile kernel per step over a
// field-major device layout.
template <typename T>
static int mode_of(Engine& E) {
  if (E.F > 1 && E.fused == 3 && E.use_sfl()) return 6;  // batches: the field-loop step
  if (E.pml) return use_persist<T>(E) ? 3 : 2;   // complex L: the one-kernel step or the persistent launch
  if (E.high_order()) return 0;                   // L^3, L^4: five kernels
  if (E.has_step4) return E.fused >= 2 ? 4 : 0;  // beta4: its one-kernel step or the five kernels
  if (use_persist<T>(E)) return 3;
  if (E.fused == 3 && E.has_step) return 2;
  return use_step<T>(E) ? 2 : (use_fused<T>(E) ? 1 : 0);
}

// State buffer holding the state before middle step k (modes 1 and 2
// alternate two buffers; mode 1 starts on psi2, mode 2 on psi).
static void* state_before(const Engine& E, int mode, int64_t k) {
  if (mode == 0) return E.psi;
  const bool odd = k % 2;
  if (mode == 1) return odd ? E.psi : E.psi2;
  return odd ? E.psi2 : E.psi;  // modes 2 to 6
}

template <typename T>
static void middle_step(const Engine& E, const DevOps<T>& d, int mode, int64_t k, double dz, double gamma,
                        hipStream_t st) {
  if (mode == 0) {
    z_step<T>(E, d, dz, gamma, dz, st);
  } else if (mode == 1) {
    fused_mid<T>(E, d, E.tiles<T>(), state_before(E, 1, k), state_before(E, 1, k + 1), dz, gamma, st);
  } else if (mode == 2) {
    launch_step<T>(d, E.stp.template ops<T>(), state_before(E, 2, k), state_before(E, 2, k + 1), dz, dz, gamma,
                   E.sblock(), st);
  } else if (mode == 4) {
    launch_step_b4<T>(d, E.stp.template ops<T>(), state_before(E, 4, k), state_before(E, 4, k + 1), dz, dz, gamma,
                      E.sblock(), st);
  } else if (mode == 6) {
    launch_step_fields<T>(d, E.sfl.template ops<T>(), state_before(E, 6, k), state_before(E, 6, k + 1), dz, dz, gamma,
                          E.fblock(), st);
  } else {  // 5: unsplit RK4
    launch_unsplit<T>(d, E.stp.template ops<T>(), state_before(E, 5, k), state_before(E, 5, k + 1), dz, gamma,
                      E.sblock(), st);
  }
}

// Steps captured per graph: the tile paths alternate two state buffers, so
// their graphs hold an even number of steps and end where they start.
static int graph_steps(const Engine& E, int mode) { return mode ? std::max(2, E.spg / 2 * 2) : E.spg; }

template <typename T>
static hipGraphExec_t get_graph(Engine& E, double dz, double gamma, int mode) {
  const int tb = mode == 1 ? E.tblock() : (mode == 6 ? E.fblock() : (mode >= 2 ? E.sblock() : 0));
  for (auto& g : E.graphs)
    if (g.dz == dz && g.gamma == gamma && g.spg == E.spg && g.block == E.block && g.xcd == E.xcd &&
        g.fused == mode && g.tile_block == tb)
      return g.exec;
  const DevOps<T> d = E.ops<T>();
  hipGraph_t graph;
  HIP_OK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
  const int steps = graph_steps(E, mode);
  for (int k = 0; k < steps; ++k) middle_step<T>(E, d, mode, k, dz, gamma, E.cap);
  hipError_t le = hipGetLastError();
  HIP_OK(hipStreamEndCapture(E.cap, &graph));
  if (le != hipSuccess) fail(DEC_BPM_EHIP, std::string("launch during capture: ") + hipGetErrorString(le));
  hipGraphExec_t exec;
  HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  if (E.graphs.size() >= 16) {
    (void)hipGraphExecDestroy(E.graphs.front().exec);
    (void)hipGraphDestroy(E.graphs.front().graph);
    E.graphs.erase(E.graphs.begin());
  }
  E.graphs.push_back(GraphEntry{dz, gamma, E.spg, E.block, E.xcd, mode, tb, exec, graph});
  return exec;
}

// Entry points whose kernels take a real L refuse handles with a PML; those
// written for the Kerr response and terms up to L^2 refuse the general ones.
static void no_pml(const Engine& E, const char* what) {
  if (E.pml) fail(DEC_BPM_EINVAL, std::string(what) + ": not available on a handle with a PML (complex L)");
}

// With a PML the adjoint runs on the one-kernel step tiles only (their
// complex-weight instances); a handle without them refuses it.
static void pml_adjoint_ok(const Engine& E, const char* what) {
  if (!E.pml) return;
  const bool ok = E.dtype == DEC_BPM_C64 ? use_step_adjoint<float>(E) : use_step_adjoint<double>(E);
  if (!ok) fail(DEC_BPM_EINVAL, std::string(what) + ": a PML needs the one-kernel step tiles, which this mesh lacks");
}
static void no_general(const Engine& E, const char* what) {
  if (E.general())
    fail(DEC_BPM_EINVAL, std::string(what) + ": not available with L^3, L^4 or a non-Kerr response");
}

static void check_stability(const Engine& E, double dz) {
  const double r = (E.rho + E.dn_max) * dz;
  if (!(r <= kStabilityLimit)) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "dz * rho(H_lin) = %.4g exceeds the RK4 stability margin %.2f (rho = %.6g)", r,
                  kStabilityLimit, E.rho + E.dn_max);
    fail(DEC_BPM_EUNSTABLE, buf);
  }
}

// Every argument check runs on the host before any device work (so a rejected
// call changes nothing); a host-only handle gets through all of them and then
// reports ENODEVICE.
static void check_prop_args(const Engine& E, const void* field, double dz, int64_t n_steps, double gamma) {
  if (!field) fail(DEC_BPM_EINVAL, "field is NULL");
  if (reinterpret_cast<uintptr_t>(field) % E.cplx_size() != 0) fail(DEC_BPM_EINVAL, "field is misaligned");
  if (!(dz > 0) || !std::isfinite(dz)) fail(DEC_BPM_EINVAL, "dz must be finite and > 0");
  if (n_steps < 0) fail(DEC_BPM_EINVAL, "n_steps must be >= 0");
  if (!std::isfinite(gamma)) fail(DEC_BPM_EINVAL, "gamma must be finite");
  check_stability(E, dz);
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
}

template <typename T>
static hipError_t run_persist(Engine& E, const TileOps<T>& tl, void* b0, void* b1, int32_t* flags, int32_t n,
                              double dz, double gamma, hipStream_t st, int body, const PersistIO& io) {
  const DevOps<T> d = E.ops<T>();
  auto launch = [&](bool coop) {
    return launch_persist<T>(d, tl, E.nb_ptr, E.nb_list, b0, b1, flags, E.flag, n, E.spin_limit, dz, gamma,
                             E.pblock(), st, body, io, coop);
  };
  if (E.coop) return launch(true);
  // a stream being captured into a graph keeps the graph's order: events
  // recorded outside the capture cannot be waited on inside it
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  int dev = 0;
  if (cap != hipStreamCaptureStatusNone || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 ||
      !g_porder[dev].ev)
    return launch(false);
  PersistOrder& o = g_porder[dev];
  std::lock_guard<std::mutex> lock(o.mu);
  if (o.has && o.last != st) {
    const hipError_t w = hipStreamWaitEvent(st, o.ev, 0);
    if (w != hipSuccess) return w;
  }
  const hipError_t e = launch(false);
  if (e != hipSuccess) return e;
  o.last = st;
  o.has = true;
  return hipEventRecord(o.ev, st);
}

// Flag base of a persistent launch of n steps (it publishes at most
// base + n + 1).  The flags are cleared only when the count would pass 2^30
// or another kernel has used them.
static PersistIO persist_io(Engine& E, int64_t n, hipStream_t st) {
  if (E.pepoch > (int32_t(1) << 30) - int32_t(std::min<int64_t>(n, int64_t(1) << 29)) - 2) {
    launch_zero_i32(E.ptiles().n_tiles, E.pflags, st);
    E.pepoch = 0;
  }
  PersistIO io;
  io.base = E.pepoch;
  E.pepoch += int32_t(n) + 2;
  return io;
}

// Whether work on the stream is being captured into a graph.
static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
}

// Middle steps (merged NL(dz)) through graph replays, then the remainder
// eagerly (all eagerly on a stream being captured: the caller's graph holds
// the launches); returns the buffer holding the state.
template <typename T>
static void* run_middle(Engine& E, int64_t count, double dz, double gamma, hipStream_t st, int mode = -1) {
  const DevOps<T> d = E.ops<T>();
  if (mode < 0) mode = mode_of<T>(E);
  // a captured graph takes one kernel per step: the persistent flags grow from call to call
  const bool cap = capturing(st);
  if (mode == 3 && cap) mode = 2;
  // unsplit RK4 on the resident tiles; not on complex128's own persistent tiles, where the
  // unsplit body's register spills make it slower than one tile kernel per step
  if (mode == 5 && E.fused == 3 && !E.pst_own && !cap && persist_fits<T>(E, 1)) {
    const int64_t chunk = int64_t(1) << 30;
    for (int64_t done = 0; done < count; done += chunk) {
      const int32_t k = int32_t(std::min(chunk, count - done));
      void* b0 = state_before(E, 5, done);
      void* b1 = b0 == E.psi ? E.psi2 : E.psi;
      hipError_t e = run_persist<T>(E, E.ptiles().template ops<T>(), b0, b1, E.pflags, k, dz, gamma, st, 1,
                                    persist_io(E, k, st));
      if (e != hipSuccess) fail(DEC_BPM_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
    }
    return state_before(E, 5, count);
  }
  if (mode == 3) {
    const int64_t chunk = int64_t(1) << 30;  // steps per launch (the parity of each chunk start is even)
    for (int64_t done = 0; done < count; done += chunk) {
      const int32_t k = int32_t(std::min(chunk, count - done));
      void* b0 = state_before(E, 3, done);
      void* b1 = b0 == E.psi ? E.psi2 : E.psi;
      hipError_t e = run_persist<T>(E, E.ptiles().template ops<T>(), b0, b1, E.pflags, k, dz, gamma, st, 0,
                                    persist_io(E, k, st));
      if (e != hipSuccess) fail(DEC_BPM_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
    }
    return state_before(E, 3, count);
  }
  const int gs = graph_steps(E, mode);
  int64_t done = 0;
  if (E.spg > 1 && count >= gs && !cap) {
    hipGraphExec_t ex = get_graph<T>(E, dz, gamma, mode);
    for (; done + gs <= count; done += gs) HIP_OK(hipGraphLaunch(ex, st));
  }
  for (; done < count; ++done) middle_step<T>(E, d, mode, done, dz, gamma, st);
  return state_before(E, mode, count);
}

// The caller's field into device order (psi), and a device-order state back.
template <typename T>
static void field_in(const Engine& E, const DevOps<T>& d, const void* field, void* dst, hipStream_t st) {
  if (E.bcbase)
    launch_bperm<T>(d, E.bcbase, E.bfcount, field, dst, false, nullptr, E.block, st);
  else
    launch_perm_in<T>(d, E.perm, field, dst, 0, E.block, st);
}
template <typename T>
static void field_out(const Engine& E, const DevOps<T>& d, const void* src, void* field, hipStream_t st) {
  if (E.bcbase)
    launch_bperm<T>(d, E.bcbase, E.bfcount, src, field, true, E.flag, E.block, st);
  else
    launch_perm_out<T>(d, E.perm, src, field, 0, E.flag, E.block, st);
}

template <typename T>
static void propagate_t(Engine& E, void* field, double dz, int64_t n, double gamma, hipStream_t st) {
  if (n == 0) return;
  const DevOps<T> d = E.ops<T>();
  const int B = E.block;
  int mode = mode_of<T>(E);
  // on a stream being captured into a graph, one kernel per step instead of the
  // persistent launch: its neighbour flags take values that grow from call to
  // call, which a replayed graph would not follow
  if (mode == 3 && capturing(st)) mode = 2;
  // one-field step tiles read the caller's field and write the result through the permutation
  const bool io_tiles = mode >= 2 && E.F == 1;
  if (!io_tiles && mode != 6) field_in<T>(E, d, field, E.psi, st);
  if (mode == 6) {
    // field-major device layout: NL(dz/2) of every field, n - 1 merged steps,
    // then LIN(dz) + NL(dz/2), back to the caller's layout
    const TileOps<T> tf = E.sfl.template ops<T>();
    launch_bperm<T>(d, E.bcbase, E.bfcount, field, E.psi2, false, nullptr, E.block, st, true);
    launch_kerr_fields<T>(d, tf, E.psi2, E.psi, 0.5 * dz, gamma, E.fblock(), st);
    void* cur = run_middle<T>(E, n - 1, dz, gamma, st, mode);
    void* nxt = cur == E.psi ? E.psi2 : E.psi;
    launch_step_fields<T>(d, tf, cur, nxt, dz, 0.5 * dz, gamma, E.fblock(), st);
    launch_bperm<T>(d, E.bcbase, E.bfcount, nxt, field, true, E.flag, E.block, st, true);
  } else if (mode == 1) {
    const TileOps<T> tl = E.tiles<T>();
    // NL(dz/2) + stage 1: state -> psi2, y1 -> ya
    launch_fused<T>(d, tl, FUSED_NL_S1, nullptr, E.psi, E.psi2, E.ya, nullptr, dz, 0.5 * dz, gamma, E.tblock(), st);
    void* cur = run_middle<T>(E, n - 1, dz, gamma, st, mode);
    void* nxt = cur == E.psi ? E.psi2 : E.psi;
    launch_fused<T>(d, tl, FUSED_S2_S3, E.ya, cur, nullptr, E.yb, nullptr, dz, dz, gamma, E.tblock(), st);
    launch_fused<T>(d, tl, FUSED_S4_NL, E.yb, cur, nxt, nullptr, nullptr, dz, 0.5 * dz, gamma, E.tblock(), st);
    field_out<T>(E, d, nxt, field, st);
  } else if (mode == 3 && io_tiles && n <= (int64_t(1) << 30)) {
    // the whole propagate in one persistent launch: NL(dz/2) of the caller's
    // field, n - 1 merged steps, then LIN(dz) + NL(dz/2) into the caller's field
    PersistIO io = persist_io(E, n, st);
    io.in = field;
    io.out = field;
    io.perm = E.perm;
    io.tau_first = io.tau_last = 0.5 * dz;
    const hipError_t e =
        run_persist<T>(E, E.ptiles().template ops<T>(), E.psi, E.psi2, E.pflags, int32_t(n), dz, gamma, st, 0, io);
    if (e != hipSuccess) fail(DEC_BPM_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
  } else if (io_tiles) {
    // NL(dz/2) of the caller's field into psi (on the step tiles: the same
    // per-row arithmetic as the persistent launch), n-1 merged steps, then
    // LIN(dz) + NL(dz/2) straight into the caller's field
    launch_kerr_tile<T>(d, E.stp.template ops<T>(), field, E.perm, E.psi, 0.5 * dz, gamma, E.sblock(), st);
    void* cur = run_middle<T>(E, n - 1, dz, gamma, st, mode);
    if (mode == 4)
      launch_step_b4<T>(d, E.stp.template ops<T>(), cur, field, dz, 0.5 * dz, gamma, E.sblock(), st, E.perm, E.flag);
    else
      launch_step<T>(d, E.stp.template ops<T>(), cur, field, dz, 0.5 * dz, gamma, E.sblock(), st, E.perm, E.flag);
  } else if (mode >= 2) {  // batched step tiles
    launch_prep_s<T>(d, E.psi, E.s, 0.5 * dz, B, st);
    launch_kerr<T>(d, E.psi, E.psi, E.s, 0.5 * dz, gamma, B, st);
    void* cur = run_middle<T>(E, n - 1, dz, gamma, st, mode);
    void* nxt = cur == E.psi ? E.psi2 : E.psi;
    launch_step<T>(d, E.stp.template ops<T>(), cur, nxt, dz, 0.5 * dz, gamma, E.sblock(), st);
    field_out<T>(E, d, nxt, field, st);
  } else {
    launch_prep_s<T>(d, E.psi, E.s, 0.5 * dz, B, st);
    do_kerr<T>(E, d, E.psi, E.psi, E.s, 0.5 * dz, gamma, st);
    run_middle<T>(E, n - 1, dz, gamma, st, mode);
    z_step<T>(E, d, dz, gamma, 0.5 * dz, st);
    field_out<T>(E, d, E.psi, field, st);
  }
  check_launch();
}

// ---- the entry point that allocates nothing ----
// dec_bpm_propagate_noalloc keeps its two state buffers and the persistent
// launch's neighbour flags in this file-scope array instead of the handle's
// buffers.  Each device holds its own copy for the life of the process, and
// every call on a device shares it.  In host code the array's name is only a
// host-side stand-in: kernels get the device address that hipGetSymbolAddress
// returned for the current device, looked up once per device.
constexpr size_t kScratchBytes = size_t(12) << 20;
constexpr size_t kScratchFlagBytes = size_t(64) << 10;  // flags of up to 16384 tiles
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[64] = {};

static unsigned char* scratch_address() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(DEC_BPM_EINVAL, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch_dev[dev]);
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Argument checks of the no-allocation variant beyond dec_bpm_propagate's.
static void check_noalloc(const Engine& E) {
  if (E.F != 1 || !(E.has_step || E.has_step4))
    fail(DEC_BPM_EINVAL,
         "dec_bpm_propagate_noalloc runs the one-field step tiles only (not for rows of more than 12 neighbours, "
         "L^3 or L^4)");
  const size_t need = 2 * round256(size_t(E.n_rows) * E.cplx_size());
  if (need > kScratchBytes - kScratchFlagBytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "dec_bpm_propagate_noalloc: the state needs %zu bytes; the static scratch holds %zu",
                  need, kScratchBytes - kScratchFlagBytes);
    fail(DEC_BPM_EINVAL, buf);
  }
  if (size_t(E.ptiles().n_tiles) * sizeof(int32_t) > kScratchFlagBytes)
    fail(DEC_BPM_EINVAL, "dec_bpm_propagate_noalloc: too many tiles for the static flag area");
}

// dec_bpm_propagate on the static scratch: the persistent launch (mode 3) or
// one tile kernel per step, launched directly (no graph), no allocation.
template <typename T>
static void propagate_noalloc_t(Engine& E, void* field, double dz, int64_t n, double gamma, hipStream_t st) {
  if (n == 0) return;
  const DevOps<T> d = E.ops<T>();
  unsigned char* base = scratch_address();
  int32_t* flags = reinterpret_cast<int32_t*>(base);
  void* b0 = base + kScratchFlagBytes;
  void* b1 = base + kScratchFlagBytes + round256(size_t(E.n_rows) * E.cplx_size());
  const int mode = mode_of<T>(E);
  if (mode == 3 && n <= (int64_t(1) << 30)) {
    launch_zero_i32(E.ptiles().n_tiles, flags, st);  // a kernel, not a memset (safe inside captured graphs)
    PersistIO io;
    io.in = field;
    io.out = field;
    io.perm = E.perm;
    io.tau_first = io.tau_last = 0.5 * dz;
    const hipError_t e =
        run_persist<T>(E, E.ptiles().template ops<T>(), b0, b1, flags, int32_t(n), dz, gamma, st, 0, io);
    if (e != hipSuccess) fail(DEC_BPM_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
  } else {
    const TileOps<T> ts = E.stp.template ops<T>();
    launch_kerr_tile<T>(d, ts, field, E.perm, b0, 0.5 * dz, gamma, E.sblock(), st);
    void* cur = b0;
    void* nxt = b1;
    for (int64_t k = 0; k < n; ++k) {
      const bool last = k == n - 1;
      void* out = last ? field : nxt;
      const double tau = last ? 0.5 * dz : dz;
      if (E.has_step4)
        launch_step_b4<T>(d, ts, cur, out, dz, tau, gamma, E.sblock(), st, last ? E.perm : nullptr, E.flag);
      else
        launch_step<T>(d, ts, cur, out, dz, tau, gamma, E.sblock(), st, last ? E.perm : nullptr, E.flag);
      std::swap(cur, nxt);
    }
  }
  check_launch();
}

static void propagate(Engine& E, void* field, double dz, int64_t n, double gamma, hipStream_t st) {
  if (E.dtype == DEC_BPM_C64)
    propagate_t<float>(E, field, dz, n, gamma, st);
  else
    propagate_t<double>(E, field, dz, n, gamma, st);
}

// n unsplit RK4 steps (no half steps to merge: every step is self-contained).
template <typename T>
static void propagate_unsplit_t(Engine& E, void* field, double dz, int64_t n, double gamma, hipStream_t st) {
  if (n == 0) return;
  const DevOps<T> d = E.ops<T>();
  launch_perm_in<T>(d, E.perm, field, E.psi, 0, E.block, st);
  void* cur = run_middle<T>(E, n, dz, gamma, st, 5);
  launch_perm_out<T>(d, E.perm, cur, field, 0, E.flag, E.block, st);
  check_launch();
}

// Tiles of the adaptive pair: seven halo rings (one per stage), the stage
// input and its |.|^2 double-buffered in LDS (6 reals per slot; 63 KiB in
// complex64, 100 KiB in complex128), one compute slot per thread of a
// 1024-thread workgroup in complex128, up to two in complex64.
template <typename T>
static bool ensure_dp5_tiles(Engine& E) {
  if (E.dp5_tried) return E.has_dp5;
  E.dp5_tried = true;
  if (!E.has_step || E.F != 1 || E.adj.arp.empty()) return false;
  const size_t lds_max = sizeof(T) == 8 ? 100 * 1024 : 63 * 1024;
  const int max_compute = (sizeof(T) == 8 || E.dp5_one_slot) ? 1024 : 2048;
  HostTiles H;
  for (int ts = E.dp5_tile; ts >= 64; ts /= 2) {
    if (!make_tiles(E.n_rows, E.adj.arp, E.adj.col, E.adj.lw, E.adj.mw, ts, 7, 7, H, true, E.sort_ring0,
                    E.adj.lwi.empty() ? nullptr : &E.adj.lwi))
      continue;
    if (size_t(H.max_slots) * 6 * sizeof(T) > lds_max || H.max_compute > max_compute) continue;
    upload_tiles<T>(E, H, E.adj.dec, E.n_rows, E.dp5);
    E.has_dp5 = true;
    break;
  }
  if (!E.has_dp5) return false;
  E.dp5ctl = static_cast<Dp5Ctl*>(E.dalloc(sizeof(Dp5Ctl)));
  E.dp5part = static_cast<double*>(E.dalloc(size_t(E.dp5.n_tiles) * 2 * sizeof(double)));
  E.dp5arr = static_cast<uint32_t*>(E.dalloc(256));
  E.dp5flags = static_cast<int32_t*>(E.dalloc(size_t(E.dp5.n_tiles) * sizeof(int32_t)));
  return true;
}

// threads per workgroup of the adaptive trial kernel: one per compute slot
// up to 1024, else two slots per thread (complex64 tiles only)
static int dp5_block(const Engine& E) {
  const int mc = E.dp5.max_compute;
  const int one = (mc + 63) / 64 * 64;
  if (one <= 1024) return std::max(64, one);
  return ((mc + 1) / 2 + 63) / 64 * 64;
}

// Whether the adaptive trial tiles can all be resident at once (the persistent
// adaptive launch), at the trial kernels' block size; the capacity is cached.
template <typename T>
static bool dp5_persist_fits(Engine& E) {
  const int blk = dp5_block(E);
  if (E.dp5_cap_block != blk) {
    E.dp5_cap = dp5_persist_capacity<T>(E.ops<T>(), E.dp5.template ops<T>(), blk);
    E.dp5_cap_block = blk;
  }
  const int64_t grid = E.xcd ? (int64_t(E.dp5.n_tiles) + 7) / 8 * 8 : E.dp5.n_tiles;
  return E.dp5_cap >= grid;
}

// Whether the whole mode iteration can run in one cooperative launch: complex64
// step tiles (complex128's persistent tiles are its own), all resident at once.
template <typename T>
static bool mode_persist_fits(Engine& E) {
  if (!E.has_persist || E.pst_own) return false;
  const int blk = E.sblock();
  if (E.mode_cap_block != blk) {
    E.mode_cap = mode_persist_capacity<T>(E.ops<T>(), E.stp.template ops<T>(), blk);
    E.mode_cap_block = blk;
  }
  const int64_t grid = E.xcd ? (int64_t(E.stp.n_tiles) + 7) / 8 * 8 : E.stp.n_tiles;
  return E.mode_cap >= grid;
}

static void ensure_mode_ctl(Engine& E) {
  if (E.modectl) return;
  E.modectl = static_cast<ModeCtl*>(E.dalloc(sizeof(ModeCtl)));
  E.modepart = static_cast<double*>(E.dalloc(size_t(E.stp.n_tiles) * 8 * sizeof(double)));
  E.modearr = static_cast<uint32_t*>(E.dalloc(256));
}

struct AdaptiveResult {
  int64_t accepted = 0, rejected = 0;
  double last_h = 0.0, z = 0.0;
  int status = 0;
};

// A graph of K back-to-back trials (each ends with its own accept/reject
// decision on the device), cached with the handle's other graphs.
template <typename T>
static hipGraphExec_t dp5_graph(Engine& E, int K, double gamma, double rtol, double atol) {
  const int blk = dp5_block(E);
  for (auto& g : E.graphs)
    if (g.fused == -K && g.gamma == gamma && g.rtol == rtol && g.atol == atol && g.block == blk && g.xcd == E.xcd)
      return g.exec;
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.dp5.template ops<T>();
  const double inv_n = 1.0 / double(E.n_rows);
  hipGraph_t graph;
  HIP_OK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < K; ++k)
    launch_dp5<T>(d, tl, E.psi, E.psi2, E.dp5ctl, E.dp5part, E.dp5arr, gamma, rtol, atol, inv_n, blk, E.cap);
  hipError_t le = hipGetLastError();
  HIP_OK(hipStreamEndCapture(E.cap, &graph));
  if (le != hipSuccess) fail(DEC_BPM_EHIP, std::string("launch during capture: ") + hipGetErrorString(le));
  hipGraphExec_t exec;
  HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  if (E.graphs.size() >= 16) {
    (void)hipGraphExecDestroy(E.graphs.front().exec);
    (void)hipGraphDestroy(E.graphs.front().graph);
    E.graphs.erase(E.graphs.begin());
  }
  GraphEntry g{0.0, gamma, 0, blk, E.xcd, -K, 0, exec, graph};
  g.rtol = rtol;
  g.atol = atol;
  E.graphs.push_back(g);
  return exec;
}

// Adaptive Dormand-Prince 5(4) from z = 0 to z_end.  Trials and decisions run
// on the device; the host enqueues them in graph-captured chunks of 8 to 512
// trials (powers of two) sized from the remaining distance at the current
// step (trials after the end return at once) and reads the controller state
// between chunks.
template <typename T>
static AdaptiveResult propagate_adaptive_t(Engine& E, void* field, double z_end, double h0, double gamma, double rtol,
                                           double atol, int64_t max_attempts, hipStream_t st) {
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.dp5.template ops<T>();
  const int blk = dp5_block(E);
  const double inv_n = 1.0 / double(E.n_rows);
  launch_perm_in<T>(d, E.perm, field, E.psi, 0, E.block, st);
  launch_dp5_init(E.dp5ctl, E.dp5arr, z_end, h0, max_attempts, 10.0, st);
  Dp5Ctl c{};
  c.h_abs = h0;
  int64_t launched = 0;
  // every seven-ring tile resident: the whole run in one cooperative launch;
  // a cooperative launch the runtime refuses (nothing was enqueued) leaves the
  // run to the per-trial kernels
  if (E.fused == 3 && dp5_persist_fits<T>(E)) {
    const hipError_t e = launch_dp5_persist<T>(d, tl, E.psi, E.psi2, E.dp5ctl, E.dp5part, E.dp5flags, E.flag,
                                               E.spin_limit, gamma, rtol, atol, inv_n, blk, st);
    if (e == hipSuccess) {
      HIP_OK(hipMemcpyAsync(&c, E.dp5ctl, sizeof(Dp5Ctl), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (!c.done) fail(DEC_BPM_EHIP, "adaptive run: a tile's wait for the others timed out");
      launched = max_attempts;
    } else {
      (void)hipGetLastError();
    }
  }
  for (; launched < max_attempts;) {
    // trials still expected at the current step size; the first chunk is short,
    // since h0 may be far from the step the controller settles on
    const double want = launched == 0 ? 8.0 : std::min((z_end - c.z) / std::max(c.h_abs, 1e-300) + 1.0, 1e9);
    const int64_t left = max_attempts - launched;
    int K = 8;
    while (K < 512 && 2 * K <= want) K *= 2;
    if (K > left) {  // the last few attempts: plain launches
      for (int64_t k = 0; k < left; ++k)
        launch_dp5<T>(d, tl, E.psi, E.psi2, E.dp5ctl, E.dp5part, E.dp5arr, gamma, rtol, atol, inv_n, blk, st);
      check_launch();
      launched += left;
    } else {
      HIP_OK(hipGraphLaunch(dp5_graph<T>(E, K, gamma, rtol, atol), st));
      launched += K;
    }
    HIP_OK(hipMemcpyAsync(&c, E.dp5ctl, sizeof(Dp5Ctl), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (c.done || launched >= max_attempts) break;
  }
  launch_perm_out<T>(d, E.perm, c.cur ? E.psi2 : E.psi, field, 0, E.flag, E.block, st);
  check_launch();
  AdaptiveResult r;
  r.accepted = c.accepted;
  r.rejected = c.rejected;
  r.last_h = c.last_h;
  r.z = c.z;
  r.status = c.done ? c.status : 1;
  return r;
}

struct ModeResult {
  double mu = 0.0, res = 0.0;
  int64_t iter = 0;
  int status = 0;
};

// A graph of K back-to-back mode iterations, cached with the other graphs
// (key: fused = -(1 << 20) - K).
template <typename T>
static hipGraphExec_t mode_graph(Engine& E, int K, double dtau, double gamma) {
  const int blk = E.sblock();
  const int key = -(1 << 20) - K;
  for (auto& g : E.graphs)
    if (g.fused == key && g.dz == dtau && g.gamma == gamma && g.block == blk && g.xcd == E.xcd) return g.exec;
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.stp.template ops<T>();
  hipGraph_t graph;
  HIP_OK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < K; ++k)
    launch_mode<T>(d, tl, E.psi, E.psi2, E.modectl, E.modepart, E.modearr, dtau, gamma, blk, E.cap);
  hipError_t le = hipGetLastError();
  HIP_OK(hipStreamEndCapture(E.cap, &graph));
  if (le != hipSuccess) fail(DEC_BPM_EHIP, std::string("launch during capture: ") + hipGetErrorString(le));
  hipGraphExec_t exec;
  HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  if (E.graphs.size() >= 16) {
    (void)hipGraphExecDestroy(E.graphs.front().exec);
    (void)hipGraphDestroy(E.graphs.front().graph);
    E.graphs.erase(E.graphs.begin());
  }
  E.graphs.push_back(GraphEntry{dtau, gamma, 0, blk, E.xcd, key, 0, exec, graph});
  return exec;
}

// Nonlinear mode iteration from the caller's field (the start) to the
// returned mode, in place.  Iterations and stopping tests run on the device
// in graph-captured chunks of 8, 16, ..., 512; the host reads the state
// between chunks and finally scales the current iterate to the power P.
template <typename T>
static ModeResult find_mode_t(Engine& E, void* field, double power, double dtau, double gamma, double tol,
                              int64_t max_iter, hipStream_t st) {
  ensure_mode_ctl(E);
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.stp.template ops<T>();
  const int blk = E.sblock();
  launch_perm_in<T>(d, E.perm, field, E.psi, 0, E.block, st);
  launch_diag<T>(d, E.psi, 0.0, E.partials, E.n_red_blocks, E.red_out, st);
  launch_mode_init(E.modectl, E.modearr, E.red_out, power, tol, max_iter, st);
  ModeCtl c{};
  int64_t launched = 0;
  int K = 8;
  // every step tile resident: the whole iteration in one cooperative launch (complex64 tiles)
  // (a refused cooperative launch enqueues nothing: the per-iteration kernels take over)
  if (E.fused == 3 && mode_persist_fits<T>(E)) {
    E.pepoch = INT32_MAX;  // the mode launch counts its iterations in the same flags
    const hipError_t e = launch_mode_persist<T>(d, tl, E.psi, E.psi2, E.modectl, E.modepart, E.pflags, E.flag,
                                                E.spin_limit, dtau, gamma, blk, st);
    if (e == hipSuccess) {
      HIP_OK(hipMemcpyAsync(&c, E.modectl, sizeof(ModeCtl), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (!c.done) fail(DEC_BPM_EHIP, "mode solver: a tile's wait for the others timed out");
      launched = max_iter;
    } else {
      (void)hipGetLastError();
    }
  }
  for (; launched < max_iter;) {
    const int64_t left = max_iter - launched;
    if (K > left) {
      for (int64_t k = 0; k < left; ++k)
        launch_mode<T>(d, tl, E.psi, E.psi2, E.modectl, E.modepart, E.modearr, dtau, gamma, blk, st);
      check_launch();
      launched += left;
    } else {
      HIP_OK(hipGraphLaunch(mode_graph<T>(E, K, dtau, gamma), st));
      launched += K;
      K = std::min(K * 2, 512);
    }
    HIP_OK(hipMemcpyAsync(&c, E.modectl, sizeof(ModeCtl), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (c.done || launched >= max_iter) break;
  }
  void* x = c.cur ? E.psi2 : E.psi;
  launch_scale<T>(E.n_rows, x, c.s, E.block, st);
  launch_perm_out<T>(d, E.perm, x, field, 0, E.flag, E.block, st);
  check_launch();
  ModeResult r;
  r.mu = c.mu;
  r.res = c.res;
  r.iter = c.iter;
  r.status = c.done ? c.status : 1;
  return r;
}

// ---- checkpointed forward and adjoint ----
struct WsLayout {
  int64_t K = 0, S = 0;
  size_t x0 = 0, ck = 0, sa = 0, sy = 0, sb = 0, ua = 0, ub = 0, acc = 0, lam = 0, sm = 0, gdn = 0, total = 0;
};

static WsLayout ws_layout(const Engine& E, int64_t n_steps, int64_t every) {
  WsLayout L;
  L.S = every > 0 ? every : std::max<int64_t>(1, int64_t(std::ceil(std::sqrt(double(std::max<int64_t>(n_steps, 1))))));
  L.K = std::max<int64_t>(1, (n_steps + L.S - 1) / L.S);
  const size_t vb = (size_t(E.n_rows) * E.cplx_size() + 255) / 256 * 256;
  size_t off = 0;
  auto take = [&](size_t count) {
    size_t o = off;
    off += count * vb;
    return o;
  };
  L.x0 = take(1);
  L.ck = take(L.K);
  L.sa = take(L.S + 1);
  L.sy = take(3 * L.S);
  L.sb = take(L.S);
  L.ua = take(1);
  L.ub = take(1);
  L.acc = take(1);
  L.lam = take(1);
  L.sm = take(1);
  L.gdn = off;
  off += (size_t(E.n_rows) * sizeof(double) + 255) / 256 * 256;
  L.total = off;
  return L;
}

// Returns whether the call recorded the last segment's stage vectors (the
// one-kernel step path does: the reverse sweep starts there without
// recomputing it; with every >= n_steps that is the whole run).
template <typename T>
static bool forward_ckpt_t(Engine& E, void* field, double dz, int64_t n, double gamma, int64_t every, char* ws,
                           hipStream_t st) {
  const WsLayout L = ws_layout(E, n, every);
  const DevOps<T> d = E.ops<T>();
  const int B = E.block;
  const size_t vb = (size_t(E.n_rows) * E.cplx_size() + 255) / 256 * 256;
  launch_perm_in<T>(d, E.perm, field, E.psi, 0, B, st);
  if (n > 0 && use_step_adjoint<T>(E)) {  // one-kernel steps
    const TileOps<T> sp = E.stp.template ops<T>();
    launch_copy<T>(E.n_rows, E.psi, ws + L.x0, B, st);
    launch_prep_s<T>(d, E.psi, E.s, 0.5 * dz, B, st);
    launch_kerr<T>(d, E.psi, E.psi, E.s, 0.5 * dz, gamma, B, st);
    launch_copy<T>(E.n_rows, E.psi, ws + L.ck, B, st);
    // the last segment's states, stage vectors and pre-Kerr states go where
    // the adjoint's recompute of that segment would put them
    const int64_t n0 = (L.K - 1) * L.S;
    auto A = [&](int64_t j) -> void* { return ws + L.sa + size_t(j) * vb; };
    auto Y = [&](int64_t j, int k) -> void* { return ws + L.sy + size_t(3 * (j - 1) + k) * vb; };
    auto Bv = [&](int64_t j) -> void* { return ws + L.sb + size_t(j - 1) * vb; };
    void* cur = E.psi;
    void* nxt = E.psi2;
    for (int64_t k = 1; k <= n; ++k) {
      const double tau = k < n ? dz : 0.5 * dz;
      if (k > n0) {
        const int64_t j = k - n0;
        launch_step_rec<T>(d, sp, cur, A(j), Y(j, 0), Y(j, 1), Y(j, 2), Bv(j), dz, tau, gamma, E.sblock(), st);
        cur = A(j);
        continue;
      }
      launch_step<T>(d, sp, cur, nxt, dz, tau, gamma, E.sblock(), st);
      std::swap(cur, nxt);
      if (k % L.S == 0 && k / L.S < L.K) launch_copy<T>(E.n_rows, cur, ws + L.ck + size_t(k / L.S) * vb, B, st);
    }
    launch_perm_out<T>(d, E.perm, cur, field, 0, E.flag, B, st);
    check_launch();
    return true;
  }
  if (n > 0 && E.has_tiles && E.fused != 0) {
    const TileOps<T> tl = E.tiles<T>();
    const int TB = E.tblock();
    launch_copy<T>(E.n_rows, E.psi, ws + L.x0, B, st);
    launch_fused<T>(d, tl, FUSED_NL_S1, nullptr, E.psi, E.psi2, E.ya, nullptr, dz, 0.5 * dz, gamma, TB, st);
    launch_copy<T>(E.n_rows, E.psi2, ws + L.ck, B, st);
    void* cur = E.psi2;
    void* nxt = E.psi;
    for (int64_t k = 1; k <= n; ++k) {
      launch_fused<T>(d, tl, FUSED_S2_S3, E.ya, cur, nullptr, E.yb, nullptr, dz, dz, gamma, TB, st);
      if (k < n)
        launch_fused<T>(d, tl, FUSED_S4_NL_S1, E.yb, cur, nxt, E.ya, nullptr, dz, dz, gamma, TB, st);
      else
        launch_fused<T>(d, tl, FUSED_S4_NL, E.yb, cur, nxt, nullptr, nullptr, dz, 0.5 * dz, gamma, TB, st);
      std::swap(cur, nxt);
      if (k % L.S == 0 && k / L.S < L.K) launch_copy<T>(E.n_rows, cur, ws + L.ck + size_t(k / L.S) * vb, B, st);
    }
    launch_perm_out<T>(d, E.perm, cur, field, 0, E.flag, B, st);
    check_launch();
    return false;
  }
  if (n > 0) {
    launch_copy<T>(E.n_rows, E.psi, ws + L.x0, B, st);
    launch_prep_s<T>(d, E.psi, E.s, 0.5 * dz, B, st);
    launch_kerr<T>(d, E.psi, E.psi, E.s, 0.5 * dz, gamma, B, st);
    launch_copy<T>(E.n_rows, E.psi, ws + L.ck, B, st);
    for (int64_t k = 1; k <= n; ++k) {
      z_step<T>(E, d, dz, gamma, k < n ? dz : 0.5 * dz, st);
      if (k % L.S == 0 && k / L.S < L.K) launch_copy<T>(E.n_rows, E.psi, ws + L.ck + size_t(k / L.S) * vb, B, st);
    }
  }
  launch_perm_out<T>(d, E.perm, E.psi, field, 0, E.flag, B, st);
  check_launch();
  return false;
}

template <typename T>
static void adjoint_t(Engine& E, const void* grad_out, double dz, int64_t n, double gamma, int64_t every, char* ws,
                      void* grad0, double* grad_dn, hipStream_t st) {
  const WsLayout L = ws_layout(E, n, every);
  const DevOps<T> d = E.ops<T>();
  const int B = E.block;
  const size_t vb = (size_t(E.n_rows) * E.cplx_size() + 255) / 256 * 256;
  void* lam = ws + L.lam;
  void* acc = ws + L.acc;
  void* ua = ws + L.ua;
  void* ub = ws + L.ub;
  void* sm = ws + L.sm;
  double* gdn = reinterpret_cast<double*>(ws + L.gdn);
  // lambda = H0^{-1} g in device order
  launch_perm_in<T>(d, E.perm, grad_out, lam, 1, B, st);
  launch_zero_f64(E.n_rows, gdn, B, st);
  auto A = [&](int64_t j) -> void* { return ws + L.sa + size_t(j) * vb; };
  auto Y = [&](int64_t j, int k) -> void* { return ws + L.sy + size_t(3 * (j - 1) + k) * vb; };
  auto Bv = [&](int64_t j) -> void* { return ws + L.sb + size_t(j - 1) * vb; };
  for (int64_t seg = L.K - 1; seg >= 0 && n > 0; --seg) {
    const int64_t n0 = seg * L.S, n1 = std::min(n, (seg + 1) * L.S), m = n1 - n0;
    // recompute the segment from its checkpoint, keeping every stage vector
    launch_copy<T>(E.n_rows, ws + L.ck + size_t(seg) * vb, A(0), B, st);
    for (int64_t j = 1; j <= m; ++j) {
      const double tau = (n0 + j < n) ? dz : 0.5 * dz;
      lin_step<T>(E, d, A(j - 1), Bv(j), Y(j, 0), Y(j, 1), Y(j, 2), dz, E.s, tau, st);
      launch_kerr<T>(d, Bv(j), A(j), E.s, tau, gamma, B, st);
    }
    // reverse sweep
    for (int64_t j = m; j >= 1; --j) {
      const double tau = (n0 + j < n) ? dz : 0.5 * dz;
      launch_adj_prep<T>(d, Bv(j), A(j), lam, sm, tau, gamma, B, st);
      launch_adj_kerr<T>(d, Bv(j), lam, sm, lam, tau, gamma, B, st);
      // reverse Horner chain of LIN(dz): links with (coef, cdn, forward vector)
      const void* uin[4] = {lam, ua, ub, ua};
      void* uout[4] = {ua, ub, ua, nullptr};
      const void* yf[4] = {Y(j, 2), Y(j, 1), Y(j, 0), A(j - 1)};
      const double co[4] = {-dz, -dz / 2, -dz / 3, -dz / 4};
      const double cd[4] = {dz, dz / 2, dz / 3, dz / 4};
      for (int k = 0; k < 4; ++k) {
        const void* t = nullptr;
        if (E.beta4 != 0.0) {
          launch_lap<T>(d, uin[k], E.t, B, st);
          t = E.t;
        }
        launch_adj_stage<T>(d, uin[k], t, uout[k], acc, k == 0, yf[k], co[k], cd[k], gdn, B, st);
      }
      std::swap(lam, acc);
    }
  }
  if (n > 0) {
    // first half step NL(dz/2) of the run: x0 -> a_0 (checkpoint 0)
    launch_adj_prep<T>(d, ws + L.x0, ws + L.ck, lam, sm, 0.5 * dz, gamma, B, st);
    launch_adj_kerr<T>(d, ws + L.x0, lam, sm, lam, 0.5 * dz, gamma, B, st);
  }
  launch_perm_out<T>(d, E.perm, lam, grad0, 1, nullptr, B, st);
  if (grad_dn) launch_gdn_out(E.n_rows, E.perm, gdn, grad_dn, B, st);
  check_launch();
}

// Adjoint on the fused tile kernels: each segment is recomputed with two
// recording tile launches per step (stages 2+3 keeping y2; stage 4 + Kerr +
// next stage 1 keeping the pre-Kerr state), then swept back with two adjoint
// tile launches per step.
template <typename T>
static void adjoint_step_t(Engine& E, const void* grad_out, double dz, int64_t n, double gamma, int64_t every,
                           char* ws, void* grad0, double* grad_dn, bool last_recorded, hipStream_t st) {
  const WsLayout L = ws_layout(E, n, every);
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> sp = E.stp.template ops<T>();
  const int B = E.block, SB = E.sblock();
  const size_t vb = (size_t(E.n_rows) * E.cplx_size() + 255) / 256 * 256;
  void* lam = ws + L.lam;
  void* other = ws + L.ua;
  void* sm = ws + L.sm;
  double* gdn = reinterpret_cast<double*>(ws + L.gdn);
  launch_perm_in<T>(d, E.perm, grad_out, lam, 1, B, st);
  launch_zero_f64(E.n_rows, gdn, B, st);
  auto Y = [&](int64_t j, int k) -> void* { return ws + L.sy + size_t(3 * (j - 1) + k) * vb; };
  auto Bv = [&](int64_t j) -> void* { return ws + L.sb + size_t(j - 1) * vb; };
  for (int64_t seg = L.K - 1; seg >= 0 && n > 0; --seg) {
    const int64_t n0 = seg * L.S, n1 = std::min(n, (seg + 1) * L.S), m = n1 - n0;
    char* ck = ws + L.ck + size_t(seg) * vb;
    auto A = [&](int64_t j) -> void* { return j == 0 ? static_cast<void*>(ck) : ws + L.sa + size_t(j) * vb; };
    // recompute the segment, recording the stage vectors (the forward call
    // recorded the last one)
    for (int64_t j = 1; j <= m && !(last_recorded && seg == L.K - 1); ++j)
      launch_step_rec<T>(d, sp, A(j - 1), A(j), Y(j, 0), Y(j, 1), Y(j, 2), Bv(j), dz, (n0 + j < n) ? dz : 0.5 * dz,
                         gamma, SB, st);
    for (int64_t j = m; j >= 1; --j) {
      launch_step_adj<T>(d, sp, lam, A(j), Bv(j), Y(j, 2), Y(j, 1), Y(j, 0), A(j - 1), other, gdn, dz,
                         (n0 + j < n) ? dz : 0.5 * dz, gamma, E.sig, SB, st);
      std::swap(lam, other);
    }
  }
  if (n > 0) {
    // first half step NL(dz/2) of the run: x0 -> a_0 (checkpoint 0)
    launch_adj_prep<T>(d, ws + L.x0, ws + L.ck, lam, sm, 0.5 * dz, gamma, B, st);
    launch_adj_kerr<T>(d, ws + L.x0, lam, sm, lam, 0.5 * dz, gamma, B, st);
  }
  launch_perm_out<T>(d, E.perm, lam, grad0, 1, nullptr, B, st);
  if (grad_dn) launch_gdn_out(E.n_rows, E.perm, gdn, grad_dn, B, st);
  check_launch();
}

template <typename T>
static bool adjoint_fused_ok(const Engine& E) {
  return E.has_tiles && E.fused != 0 && size_t(E.tl.max_slots) * 4 * 2 * sizeof(T) <= 64 * 1024;
}

template <typename T>
static void adjoint_fused_t(Engine& E, const void* grad_out, double dz, int64_t n, double gamma, int64_t every,
                            char* ws, void* grad0, double* grad_dn, hipStream_t st) {
  const WsLayout L = ws_layout(E, n, every);
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.tiles<T>();
  const int B = E.block, TB = E.tblock();
  const size_t vb = (size_t(E.n_rows) * E.cplx_size() + 255) / 256 * 256;
  void* lam = ws + L.lam;
  void* acc = ws + L.acc;
  void* ua = ws + L.ua;
  void* sm = ws + L.sm;
  double* gdn = reinterpret_cast<double*>(ws + L.gdn);
  launch_perm_in<T>(d, E.perm, grad_out, lam, 1, B, st);
  launch_zero_f64(E.n_rows, gdn, B, st);
  auto Y = [&](int64_t j, int k) -> void* { return ws + L.sy + size_t(3 * (j - 1) + k) * vb; };
  auto Bv = [&](int64_t j) -> void* { return ws + L.sb + size_t(j - 1) * vb; };
  for (int64_t seg = L.K - 1; seg >= 0 && n > 0; --seg) {
    const int64_t n0 = seg * L.S, n1 = std::min(n, (seg + 1) * L.S), m = n1 - n0;
    char* ck = ws + L.ck + size_t(seg) * vb;
    auto A = [&](int64_t j) -> void* { return j == 0 ? static_cast<void*>(ck) : ws + L.sa + size_t(j) * vb; };
    launch_stage<T>(d, A(0), nullptr, A(0), Y(1, 0), dz / 4, nullptr, 0.0, B, st);
    for (int64_t j = 1; j <= m; ++j) {
      const double tau = (n0 + j < n) ? dz : 0.5 * dz;
      launch_fused<T>(d, tl, FUSED_S2_S3, Y(j, 0), A(j - 1), nullptr, Y(j, 2), Y(j, 1), dz, dz, gamma, TB, st);
      if (j < m)
        launch_fused<T>(d, tl, FUSED_S4_NL_S1, Y(j, 2), A(j - 1), A(j), Y(j + 1, 0), Bv(j), dz, tau, gamma, TB, st);
      else
        launch_fused<T>(d, tl, FUSED_S4_NL, Y(j, 2), A(j - 1), A(j), nullptr, Bv(j), dz, tau, gamma, TB, st);
    }
    for (int64_t j = m; j >= 1; --j) {
      const double tau = (n0 + j < n) ? dz : 0.5 * dz;
      launch_fused_adj<T>(d, tl, 1, lam, A(j), Bv(j), Y(j, 2), Y(j, 1), Y(j, 0), ua, acc, gdn, dz, tau, gamma, TB,
                          st);
      launch_fused_adj<T>(d, tl, 2, ua, A(j - 1), nullptr, nullptr, nullptr, nullptr, lam, acc, gdn, dz, tau, gamma,
                          TB, st);
    }
  }
  if (n > 0) {
    // first half step NL(dz/2) of the run: x0 -> a_0 (checkpoint 0)
    launch_adj_prep<T>(d, ws + L.x0, ws + L.ck, lam, sm, 0.5 * dz, gamma, B, st);
    launch_adj_kerr<T>(d, ws + L.x0, lam, sm, lam, 0.5 * dz, gamma, B, st);
  }
  launch_perm_out<T>(d, E.perm, lam, grad0, 1, nullptr, B, st);
  if (grad_dn) launch_gdn_out(E.n_rows, E.perm, gdn, grad_dn, B, st);
  check_launch();
}

// ---- kernel timing with HIP events (graph-captured back-to-back launches) ----
template <typename T>
static void time_kernels_t(Engine& E, double dz, double gamma, int reps, double* ms, double* bytes, hipStream_t st) {
  const DevOps<T> d = E.ops<T>();
  const TileOps<T> tl = E.tiles<T>();
  const int B = E.block;
  const double sr = sizeof(T), sc = 2 * sizeof(T);
  const double nF = double(E.n_rows) * E.F, nr = double(E.n_rows);
  const double mat = double(E.nnz_off) * (4.0 + sr);
  const double mat_lm = double(E.nnz_off) * (4.0 + (E.mw ? 2 : 1) * sr);  // L and M share the pattern
  double by[DEC_BPM_NUM_KERNELS];
  by[DEC_BPM_K_KERR] = (E.mw ? mat : 0.0) + nr * 2 * sr + nF * (sr + 2 * sc);
  by[DEC_BPM_K_STAGE] = mat + nr * sr + nF * 3 * sc;
  by[DEC_BPM_K_LAP] = mat + nF * 2 * sc;
  // fused kernels, counted once per owned row (halo recompute is overhead, not algorithmic):
  // A reads y3, psi, v, w, M_pp and both operators; writes psi'' and y1.  B reads y1, psi, v, L; writes y3.
  // The one-kernel step reads psi, v, w, M_pp and both operators and writes psi.
  by[DEC_BPM_K_TILE_A] = mat_lm + nr * 3 * sr + nr * 4 * sc;
  by[DEC_BPM_K_TILE_B] = mat + nr * sr + nr * 3 * sc;
  by[DEC_BPM_K_STEP] = mat_lm + nr * 3 * sr + nF * 2 * sc;
  // persistent stepping, per z step: the same algorithmic bytes as the one-kernel step (the
  // implementation keeps the operator rows on chip, the algorithm still needs them every step)
  by[DEC_BPM_K_PERSIST] = by[DEC_BPM_K_STEP];
  by[DEC_BPM_K_UNSPLIT] = by[DEC_BPM_K_STEP];  // one unsplit RK4 step: the same data
  by[DEC_BPM_K_DP5] = by[DEC_BPM_K_STEP];      // one adaptive trial: the same data
  by[DEC_BPM_K_MODE] = by[DEC_BPM_K_STEP];     // one mode iteration: the same data
  by[DEC_BPM_K_DP5_PERSIST] = by[DEC_BPM_K_STEP];
  by[DEC_BPM_K_MODE_PERSIST] = by[DEC_BPM_K_STEP];
  by[DEC_BPM_K_UNSPLIT_PERSIST] = by[DEC_BPM_K_STEP];
  launch_fill<T>(d, E.psi, 0.3, 0.1, B, st);
  launch_fill<T>(d, E.ya, 0.2, -0.1, B, st);
  launch_fill<T>(d, E.yb, 0.2, -0.1, B, st);
  if (E.psi2) launch_fill<T>(d, E.psi2, 0.3, 0.1, B, st);
  launch_prep_s<T>(d, E.psi, E.s, dz, B, st);
  HIP_OK(hipStreamSynchronize(st));
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  for (int kind = 0; kind < DEC_BPM_NUM_KERNELS; ++kind) {
    const bool tile_kind = kind == DEC_BPM_K_TILE_A || kind == DEC_BPM_K_TILE_B;
    if ((tile_kind && !E.has_tiles) || (kind == DEC_BPM_K_STEP && !E.has_step && !E.has_step4 && !E.use_sfl()) ||
        (kind == DEC_BPM_K_UNSPLIT && (!E.has_step || E.F != 1)) ||
        (kind == DEC_BPM_K_DP5 && !(E.has_step && E.F == 1 && ensure_dp5_tiles<T>(E))) ||
        (kind == DEC_BPM_K_MODE && !(E.has_step && E.F == 1)) ||
        (kind == DEC_BPM_K_MODE_PERSIST && !(E.has_step && E.F == 1 && mode_persist_fits<T>(E))) ||
        (kind == DEC_BPM_K_UNSPLIT_PERSIST && !(E.has_persist && !E.pst_own && persist_fits<T>(E, 1))) ||
        (kind == DEC_BPM_K_DP5_PERSIST &&
         !(E.has_step && E.F == 1 && ensure_dp5_tiles<T>(E) && dp5_persist_fits<T>(E))) ||
        (kind == DEC_BPM_K_PERSIST && !(E.has_persist && persist_fits<T>(E)))) {
      if (ms) ms[kind] = 0.0;
      if (bytes) bytes[kind] = 0.0;
      continue;
    }
    if (kind == DEC_BPM_K_PERSIST || kind == DEC_BPM_K_UNSPLIT_PERSIST) {  // one launch of >= 2000 steps
      const TileOps<T> sp = E.ptiles().template ops<T>();
      const int steps = std::max(reps, 2000);  // the launch's fixed cost spread thin, as in a long propagate
      const int body = kind == DEC_BPM_K_UNSPLIT_PERSIST ? 1 : 0;
      // the split body as a propagate runs it: from a caller-order field (ya) to another (yb)
      auto io = [&](int n) {
        PersistIO r = persist_io(E, n, st);
        if (body == 0) {
          r.in = E.ya;
          r.out = E.yb;
          r.perm = E.perm;
          r.tau_first = r.tau_last = 0.5 * dz;
        }
        return r;
      };
      HIP_OK(run_persist<T>(E, sp, E.psi, E.psi2, E.pflags, 2, dz, gamma, st, body, io(2)));  // warm-up
      const PersistIO timed = io(steps);
      HIP_OK(hipEventRecord(e0, st));
      HIP_OK(run_persist<T>(E, sp, E.psi, E.psi2, E.pflags, steps, dz, gamma, st, body, timed));
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float t = 0;
      HIP_OK(hipEventElapsedTime(&t, e0, e1));
      if (ms) ms[kind] = double(t) / steps;
      if (bytes) bytes[kind] = by[kind];
      continue;
    }
    if (kind == DEC_BPM_K_DP5_PERSIST) {  // one launch of a fixed trial count, time per trial
      const TileOps<T> tp = E.dp5.template ops<T>();
      const int blk = dp5_block(E);
      const int trials = std::max(reps, 200);
      bool refused = false;  // a cooperative launch the runtime refuses: reported as 0, like an absent path
      for (int pass = 0; pass < 2 && !refused; ++pass) {  // warm-up, then timed
        const int n = pass ? trials : 2;
        launch_dp5_init(E.dp5ctl, E.dp5arr, 1e300, dz, n, 1.0, st);
        if (pass) HIP_OK(hipEventRecord(e0, st));
        refused = launch_dp5_persist<T>(d, tp, E.psi, E.psi2, E.dp5ctl, E.dp5part, E.dp5flags, E.flag, E.spin_limit,
                                        gamma, 1e-6, 1e-8, 1.0 / double(E.n_rows), blk, st) != hipSuccess;
      }
      if (refused) {
        (void)hipGetLastError();
        if (ms) ms[kind] = 0.0;
        if (bytes) bytes[kind] = by[kind];
        continue;
      }
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float t = 0;
      HIP_OK(hipEventElapsedTime(&t, e0, e1));
      if (ms) ms[kind] = double(t) / trials;
      if (bytes) bytes[kind] = by[kind];
      continue;
    }
    if (kind == DEC_BPM_K_MODE_PERSIST) {  // one launch of a fixed iteration count, time per iteration
      ensure_mode_ctl(E);
      const TileOps<T> ts = E.stp.template ops<T>();
      const int iters = std::max(reps, 200);
      bool refused = false;  // as for the adaptive run's launch
      for (int pass = 0; pass < 2 && !refused; ++pass) {  // warm-up, then timed
        launch_diag<T>(d, E.psi, 0.0, E.partials, E.n_red_blocks, E.red_out, st);
        launch_mode_init(E.modectl, E.modearr, E.red_out, 1.0, 0.0, pass ? iters : 2, st);
        if (pass) HIP_OK(hipEventRecord(e0, st));
        E.pepoch = INT32_MAX;  // the mode launch counts its iterations in the same flags
        refused = launch_mode_persist<T>(d, ts, E.psi, E.psi2, E.modectl, E.modepart, E.pflags, E.flag,
                                         E.spin_limit, dz, gamma, E.sblock(), st) != hipSuccess;
      }
      if (refused) {
        (void)hipGetLastError();
        if (ms) ms[kind] = 0.0;
        if (bytes) bytes[kind] = by[kind];
        continue;
      }
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float t = 0;
      HIP_OK(hipEventElapsedTime(&t, e0, e1));
      if (ms) ms[kind] = double(t) / iters;
      if (bytes) bytes[kind] = by[kind];
      continue;
    }
    if (kind == DEC_BPM_K_MODE) {  // iterations of step dz at power 1, no stopping test
      ensure_mode_ctl(E);
      launch_diag<T>(d, E.psi, 0.0, E.partials, E.n_red_blocks, E.red_out, st);
      launch_mode_init(E.modectl, E.modearr, E.red_out, 1.0, 0.0, int64_t(1) << 62, st);
      HIP_OK(hipStreamSynchronize(st));
    }
    if (kind == DEC_BPM_K_DP5) {  // trials of step dz (growth factor capped at 1, no end in sight)
      launch_dp5_init(E.dp5ctl, E.dp5arr, 1e300, dz, int64_t(1) << 62, 1.0, st);
      HIP_OK(hipStreamSynchronize(st));
    }
    hipGraph_t g;
    HIP_OK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < reps; ++r) {
      if (kind == DEC_BPM_K_KERR) do_kerr<T>(E, d, E.psi, E.psi, E.s, dz, gamma, E.cap);
      if (kind == DEC_BPM_K_STAGE) do_stage<T>(E, d, E.ya, nullptr, E.psi, E.yb, dz / 3, nullptr, 0.0, E.cap);
      if (kind == DEC_BPM_K_LAP) do_lap<T>(E, d, E.ya, E.yb, E.cap);
      if (kind == DEC_BPM_K_TILE_A)
        launch_fused<T>(d, tl, FUSED_S4_NL_S1, E.yb, E.psi, E.psi2, E.ya, nullptr, dz, dz, gamma, E.tblock(), E.cap);
      if (kind == DEC_BPM_K_TILE_B)
        launch_fused<T>(d, tl, FUSED_S2_S3, E.ya, E.psi, nullptr, E.yb, nullptr, dz, dz, gamma, E.tblock(), E.cap);
      if (kind == DEC_BPM_K_STEP && E.use_sfl() && (mode_of<T>(E) == 6 || !E.has_step))
        launch_step_fields<T>(d, E.sfl.template ops<T>(), r % 2 ? E.psi2 : E.psi, r % 2 ? E.psi : E.psi2, dz, dz,
                              gamma, E.fblock(), E.cap);
      else if (kind == DEC_BPM_K_STEP && E.has_step4)
        launch_step_b4<T>(d, E.stp.template ops<T>(), r % 2 ? E.psi2 : E.psi, r % 2 ? E.psi : E.psi2, dz, dz,
                          gamma, E.sblock(), E.cap);
      else if (kind == DEC_BPM_K_STEP)
        launch_step<T>(d, E.stp.template ops<T>(), r % 2 ? E.psi2 : E.psi, r % 2 ? E.psi : E.psi2, dz, dz, gamma,
                       E.sblock(), E.cap);
      if (kind == DEC_BPM_K_UNSPLIT)
        launch_unsplit<T>(d, E.stp.template ops<T>(), r % 2 ? E.psi2 : E.psi, r % 2 ? E.psi : E.psi2, dz, gamma,
                          E.sblock(), E.cap);
      if (kind == DEC_BPM_K_MODE)
        launch_mode<T>(d, E.stp.template ops<T>(), E.psi, E.psi2, E.modectl, E.modepart, E.modearr, dz, gamma,
                       E.sblock(), E.cap);
      if (kind == DEC_BPM_K_DP5)
        launch_dp5<T>(d, E.dp5.template ops<T>(), E.psi, E.psi2, E.dp5ctl, E.dp5part, E.dp5arr, gamma, 1e-6, 1e-8,
                      1.0 / double(E.n_rows), dp5_block(E), E.cap);
    }
    HIP_OK(hipStreamEndCapture(E.cap, &g));
    hipGraphExec_t ex;
    HIP_OK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    HIP_OK(hipGraphLaunch(ex, st));  // warm-up
    HIP_OK(hipEventRecord(e0, st));
    HIP_OK(hipGraphLaunch(ex, st));
    HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipEventSynchronize(e1));
    float t = 0;
    HIP_OK(hipEventElapsedTime(&t, e0, e1));
    if (ms) ms[kind] = double(t) / reps;
    if (bytes) bytes[kind] = by[kind];
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ---- autotuning ----
static std::string tune_key(const Engine& E) {
  std::ostringstream o;
  o << "n" << E.n_rows << "_e" << E.n_entries << "_F" << E.F << "_d" << E.dtype << "_b4" << (E.beta4 != 0.0) << "_nl"
    << (E.mw ? 0 : 1) << "_ts" << (E.has_tiles ? E.tile_size : 0) << "_st" << ((E.has_step || E.has_step4) ? E.step_tile : 0);
  return o.str();
}

static bool tune_cache_lookup(Engine& E) {
  const char* path = std::getenv("DEC_BPM_TUNE_CACHE");
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line, key = "\"" + tune_key(E) + "\"";
  while (std::getline(f, line)) {
    size_t p = line.find(key);
    if (p == std::string::npos) continue;
    int b = 0, s = 0, x = 1, fu = 0, tb = 256;
    if (std::sscanf(line.c_str() + p + key.size(),
                    ": {\"block\": %d, \"steps_per_graph\": %d, \"xcd\": %d, \"fused\": %d, \"tile_block\": %d}",
                    &b, &s, &x, &fu, &tb) == 5 &&
        b >= 64 && s >= 1 && tb >= 64) {
      E.block = b;
      E.spg = s;
      E.xcd = x;
      E.fused = (E.has_tiles || E.has_btiles || E.has_step || E.has_step4 || E.has_sfl) ? fu : 0;
      E.tile_block = tb;
      return true;
    }
  }
  return false;
}

static void tune_cache_store(const Engine& E) {
  const char* path = std::getenv("DEC_BPM_TUNE_CACHE");
  if (!path) return;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
      if (line.find("\"" + tune_key(E) + "\"") == std::string::npos && line.find(": {") != std::string::npos)
        lines.push_back(line);
  }
  std::ofstream f(path);
  f << "{\n";
  for (auto& l : lines) {
    std::string x = l;
    while (!x.empty() && (x.back() == ',' || x.back() == ' ')) x.pop_back();
    f << x << ",\n";
  }
  f << "  \"" << tune_key(E) << "\": {\"block\": " << E.block << ", \"steps_per_graph\": " << E.spg
    << ", \"xcd\": " << E.xcd << ", \"fused\": " << E.fused << ", \"tile_block\": " << E.tile_block << "}\n}\n";
}

template <typename T>
static void autotune_t(Engine& E, double dz, double gamma, hipStream_t st) {
  if (tune_cache_lookup(E)) return;
  const DevOps<T> d0 = E.ops<T>();
  struct Cand {
    int fused, block, tile_block, spg, xcd;
  };
  std::vector<Cand> cands;
  for (int x : {0, 1})
    for (int s : {1, 8, 32, 128}) {
      if (!E.pml)
        for (int b : {64, 128, 256, 512, 1024}) cands.push_back({0, b, E.tile_block, s, x});
      if (E.has_tiles)
        for (int tb : {128, 256, 512, 1024}) cands.push_back({1, E.block, tb, s, x});
      if (E.has_step || E.has_step4)
        for (int tb : {256, 512, 1024}) cands.push_back({2, E.block, tb, s, x});
      if (E.has_persist && s == 32)  // one launch runs every step: steps per graph do not apply
        for (int tb : {256, 512, 1024}) cands.push_back({3, E.block, tb, s, x});
      if (E.has_btiles) cands.push_back({1, E.block, E.tile_block, s, x});
      if (E.has_sfl && E.F > 1)
        for (int tb : {256, 512, 1024}) cands.push_back({3, E.block, tb, s, x});
    }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  double best = 1e300;
  Cand bc{E.fused, E.block, E.tile_block, E.spg, E.xcd};
  const int64_t steps = 128;
  for (const Cand& c : cands) {
    E.fused = c.fused;
    E.block = c.block;
    E.tile_block = c.tile_block;
    E.spg = c.spg;
    E.xcd = c.xcd;
    if (c.fused == 3 && (E.F > 1 ? !E.use_sfl() : !persist_fits<T>(E))) continue;
    launch_fill<T>(d0, E.psi, 0.3, 0.1, 256, st);
    if (E.psi2) launch_fill<T>(d0, E.psi2, 0.3, 0.1, 256, st);
    launch_fill<T>(d0, E.ya, 0.3, 0.1, 256, st);
    launch_fill<T>(d0, E.yb, 0.3, 0.1, 256, st);
    launch_prep_s<T>(d0, E.psi, E.s, dz, 256, st);
    run_middle<T>(E, graph_steps(E, mode_of<T>(E)), dz, gamma, st);  // warm-up (and graph instantiation)
    HIP_OK(hipEventRecord(e0, st));
    run_middle<T>(E, steps, dz, gamma, st);
    HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipEventSynchronize(e1));
    float t = 0;
    HIP_OK(hipEventElapsedTime(&t, e0, e1));
    if (t < best) {
      best = t;
      bc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  E.drop_graphs();
  E.fused = bc.fused;
  E.block = bc.block;
  E.tile_block = bc.tile_block;
  E.spg = bc.spg;
  E.xcd = bc.xcd;
  tune_cache_store(E);
}

}  // namespace decbpm

using decbpm::Engine;
using decbpm::Error;
using decbpm::fail;

struct dec_bpm_s {
  decbpm::Assembled A;
  dec_bpm_options opt;
  Engine E;
  ~dec_bpm_s() { E.release(); }
};

struct dec_bpm_batch_s {
  Engine E;
  int64_t n_elems = 0;  // packed complex elements in the caller's layout
  ~dec_bpm_batch_s() { E.release(); }
};

#define ABI_TRY try {
#define ABI_CATCH                                                              \
  }                                                                            \
  catch (const Error& e) {                                                     \
    decbpm::g_last_error = e.msg;                                              \
    return e.code;                                                             \
  }                                                                            \
  catch (const std::bad_alloc&) {                                              \
    decbpm::g_last_error = "host allocation failed";                           \
    return DEC_BPM_ENOMEM;                                                     \
  }                                                                            \
  catch (const std::exception& e) {                                            \
    decbpm::g_last_error = e.what();                                           \
    return DEC_BPM_EINVAL;                                                     \
  }                                                                            \
  catch (...) {                                                                \
    decbpm::g_last_error = "unknown error";                                    \
    return DEC_BPM_EINVAL;                                                     \
  }                                                                            \
  decbpm::g_last_error.clear();                                                \
  return DEC_BPM_OK;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

static dec_bpm_s* need(dec_bpm_t h) {
  if (!h) fail(DEC_BPM_EINVAL, "handle is NULL");
  return h;
}

extern "C" {

void dec_bpm_default_options(dec_bpm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->struct_size = sizeof(dec_bpm_options);
  o->dtype = DEC_BPM_C64;
  o->p1 = 0.5;
  o->beta4 = 0.0;
  o->nonlinearity = DEC_BPM_NL_DEC;
  o->reorder = 1;
  o->chi_tri = nullptr;
  o->host_only = 0;
  o->block_size = 0;
  o->steps_per_graph = 0;
}

const char* dec_bpm_last_error(void) { return decbpm::g_last_error.c_str(); }

const char* dec_bpm_version(void) { return "dec_bpm 0.1 (gfx950)"; }

int dec_bpm_create(const double* xy, int64_t n_vert, const int32_t* tri, int64_t n_tri, const double* index_tri,
                   const double* absorber_vert, const dec_bpm_options* opt, dec_bpm_t* out) {
  ABI_TRY
  if (!out) fail(DEC_BPM_EINVAL, "out is NULL");
  *out = nullptr;
  dec_bpm_options o;
  dec_bpm_default_options(&o);
  if (opt) {
    if (opt->struct_size != sizeof(dec_bpm_options)) fail(DEC_BPM_EINVAL, "dec_bpm_options.struct_size mismatch");
    o = *opt;
  }
  if (o.dtype != DEC_BPM_C64 && o.dtype != DEC_BPM_C128) fail(DEC_BPM_EINVAL, "dtype must be C64 or C128");
  if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 1024 || o.block_size % 64 != 0))
    fail(DEC_BPM_EINVAL, "block_size must be a multiple of 64 in [64, 1024]");
  if (o.steps_per_graph < 0) fail(DEC_BPM_EINVAL, "steps_per_graph must be >= 0");
  decbpm::AssemblyInput in;
  in.xy = xy;
  in.n = n_vert;
  in.tri = tri;
  in.n_tri = n_tri;
  in.index_tri = index_tri;
  in.absorber = absorber_vert;
  in.chi_tri = o.chi_tri;
  in.p1 = o.p1;
  in.beta4 = o.beta4;
  in.nonlinearity = o.nonlinearity;
  in.reorder = o.reorder != 0;
  in.pml_r0 = o.pml_r0;
  in.pml_r1 = o.pml_r1;
  in.pml_sigma = o.pml_sigma;
  in.p3 = o.p3;
  in.p4 = o.p4;
  if (o.nl_kind < DEC_BPM_N_KERR || o.nl_kind > DEC_BPM_N_CUBIC_QUINTIC) fail(DEC_BPM_EINVAL, "unknown nl_kind");
  if (o.nl_kind == DEC_BPM_N_SATURABLE && !(o.nl_param > 0.0 && std::isfinite(o.nl_param)))
    fail(DEC_BPM_EINVAL, "the saturable response needs nl_param = I_s > 0");
  if (o.nl_kind == DEC_BPM_N_CUBIC_QUINTIC && !(o.nl_param >= 0.0 && std::isfinite(o.nl_param)))
    fail(DEC_BPM_EINVAL, "the cubic-quintic response needs nl_param >= 0");
  if ((o.p3 != 0.0 || o.p4 != 0.0 || o.nl_kind != DEC_BPM_N_KERR) && o.pml_sigma > 0.0)
    fail(DEC_BPM_EINVAL, "a PML does not combine with L^3, L^4 or a non-Kerr response");
  std::unique_ptr<dec_bpm_s> h(new dec_bpm_s());
  h->A = decbpm::assemble(in);
  o.chi_tri = nullptr;  // not kept
  h->opt = o;
  Engine& E = h->E;
  E.dtype = o.dtype;
  E.F = 1;
  E.p1 = o.p1;
  E.beta4 = o.beta4;
  E.nl = o.nonlinearity;
  E.p3 = o.p3;
  E.p4 = o.p4;
  E.nk = o.nl_kind;
  E.npar = o.nl_param;
  E.rho = h->A.rho;
  E.pml = !h->A.kp_re.empty();
  if (!o.host_only) {
    decbpm::build_engine(E, {&h->A}, {o.nonlinearity == DEC_BPM_NL_LUMPED ? 1 : 0});
    if (o.block_size) E.block = o.block_size;
    if (o.steps_per_graph) E.spg = o.steps_per_graph;
  } else {
    E.n_rows = h->A.n;
  }
  *out = h.release();
  ABI_CATCH
}

void dec_bpm_destroy(dec_bpm_t h) { delete h; }

int dec_bpm_sizes(dec_bpm_t h, int64_t* n_vert, int64_t* n_tri, int64_t* n_edge, int64_t* nnz) {
  ABI_TRY
  need(h);
  if (n_vert) *n_vert = h->A.n;
  if (n_tri) *n_tri = h->A.n_tri;
  if (n_edge) *n_edge = h->A.n_edge;
  if (nnz) *nnz = h->A.rp.empty() ? 0 : h->A.rp.back();
  ABI_CATCH
}

int dec_bpm_spectral_radius(dec_bpm_t h, double* rho) {
  ABI_TRY
  need(h);
  if (!rho) fail(DEC_BPM_EINVAL, "rho is NULL");
  *rho = h->E.rho + h->E.dn_max;
  ABI_CATCH
}

int dec_bpm_export_operators(dec_bpm_t h, double* h0, double* v, double* w, int64_t* nnz, int64_t* row_ptr,
                             int32_t* col, double* kval, double* mval) {
  ABI_TRY
  need(h);
  const auto& A = h->A;
  if (nnz) *nnz = A.rp.back();
  if (h0) std::copy(A.h0.begin(), A.h0.end(), h0);
  if (v) std::copy(A.v.begin(), A.v.end(), v);
  if (w) std::copy(A.w.begin(), A.w.end(), w);
  if (row_ptr) std::copy(A.rp.begin(), A.rp.end(), row_ptr);
  if (col) std::copy(A.col.begin(), A.col.end(), col);
  if (kval) std::copy(A.k.begin(), A.k.end(), kval);
  if (mval) std::copy(A.qdq.begin(), A.qdq.end(), mval);
  ABI_CATCH
}

int dec_bpm_vertex_tiles(dec_bpm_t h, int32_t* tile, int32_t* rows_per_tile) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  int ts = -1;
  if (E.on_device) {
    const int mode = E.dtype == DEC_BPM_C64 ? decbpm::mode_of<float>(E) : decbpm::mode_of<double>(E);
    if (mode == 3) ts = E.ptiles().TS;
    else if (mode >= 2) ts = E.stp.TS;
    else if (mode == 1) ts = E.tl.TS;
  }
  if (rows_per_tile) *rows_per_tile = ts;
  if (tile)
    for (int64_t i = 0; i < h->A.n; ++i) tile[i] = ts > 0 ? h->A.iperm[i] / ts : -1;
  ABI_CATCH
}

int dec_bpm_export_pml(dec_bpm_t h, double* h0p, double* kp) {
  ABI_TRY
  need(h);
  const decbpm::Assembled& A = h->A;
  if (A.kp_re.empty()) fail(DEC_BPM_EINVAL, "the handle has no PML");
  if (h0p)
    for (int64_t p = 0; p < A.n; ++p) {
      h0p[2 * p] = A.h0p_re[p];
      h0p[2 * p + 1] = A.h0p_im[p];
    }
  if (kp)
    for (size_t e = 0; e < A.kp_re.size(); ++e) {
      kp[2 * e] = A.kp_re[e];
      kp[2 * e + 1] = A.kp_im[e];
    }
  ABI_CATCH
}

int dec_bpm_set_index_perturbation(dec_bpm_t h, const double* dn_dev, void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  double mx = 0.0;
  uint64_t digest = 0;
  if (dn_dev) {
    std::vector<double> host(E.n_rows);
    HIP_OK(hipMemcpyAsync(host.data(), dn_dev, E.n_rows * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (double x : host) {
      if (!std::isfinite(x)) fail(DEC_BPM_EINVAL, "index perturbation has a non-finite entry");
      mx = std::max(mx, std::fabs(x));
    }
    // FNV-1a over the values' bytes; 0 is kept for "none"
    digest = 1469598103934665603ull;
    const unsigned char* b = reinterpret_cast<const unsigned char*>(host.data());
    for (size_t i = 0; i < host.size() * sizeof(double); ++i) digest = (digest ^ b[i]) * 1099511628211ull;
    if (digest == 0) digest = 1;
  }
  if (E.dtype == DEC_BPM_C64)
    decbpm::launch_set_v<float>(E.n_rows, static_cast<const float*>(E.v0), dn_dev, E.perm, static_cast<float*>(E.v),
                                256, st);
  else
    decbpm::launch_set_v<double>(E.n_rows, static_cast<const double*>(E.v0), dn_dev, E.perm,
                                 static_cast<double*>(E.v), 256, st);
  decbpm::check_launch();
  HIP_OK(hipStreamSynchronize(st));
  E.dn_max = mx;
  E.dn_digest = digest;
  ABI_CATCH
}

int dec_bpm_apply(dec_bpm_t h, int op, const void* x, void* y, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_pml(h->E, "dec_bpm_apply");
  Engine& E = h->E;
  if (!x || !y || x == y) fail(DEC_BPM_EINVAL, "x and y must be distinct non-NULL device vectors");
  if (op < DEC_BPM_OP_L || op > DEC_BPM_OP_H) fail(DEC_BPM_EINVAL, "unknown operator");
  if (op == DEC_BPM_OP_H && (E.p3 != 0.0 || E.p4 != 0.0))
    fail(DEC_BPM_EINVAL, "dec_bpm_apply(H): not available with L^3 or L^4 terms");
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const decbpm::DevOps<T> d = E.ops<T>();
    const int B = E.block;
    decbpm::launch_perm_in<T>(d, E.perm, x, E.ya, 0, B, st);
    decbpm::launch_lap<T>(d, E.ya, E.yb, B, st);  // yb = L x
    void* res = E.yb;
    if (op == DEC_BPM_OP_L2) {
      decbpm::launch_lap<T>(d, E.yb, E.psi, B, st);
      res = E.psi;
    } else if (op == DEC_BPM_OP_H) {
      void* t2 = nullptr;
      if (E.beta4 != 0.0) {
        decbpm::launch_lap<T>(d, E.yb, E.t, B, st);
        t2 = E.t;
      }
      decbpm::launch_hcombine<T>(d, E.ya, E.yb, t2, E.psi, B, st);
      res = E.psi;
    }
    decbpm::launch_perm_out<T>(d, E.perm, res, y, 0, nullptr, B, st);
  };
  if (E.dtype == DEC_BPM_C64)
    run(float{});
  else
    run(double{});
  decbpm::check_launch();
  ABI_CATCH
}

int dec_bpm_kerr_step(dec_bpm_t h, void* field, double tau, double gamma, void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!field) fail(DEC_BPM_EINVAL, "field is NULL");
  if (!(tau >= 0) || !std::isfinite(tau) || !std::isfinite(gamma)) fail(DEC_BPM_EINVAL, "bad tau or gamma");
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const decbpm::DevOps<T> d = E.ops<T>();
    decbpm::launch_perm_in<T>(d, E.perm, field, E.psi, 0, E.block, st);
    decbpm::launch_prep_s<T>(d, E.psi, E.s, tau, E.block, st);
    decbpm::launch_kerr<T>(d, E.psi, E.psi, E.s, tau, gamma, E.block, st);
    decbpm::launch_perm_out<T>(d, E.perm, E.psi, field, 0, E.flag, E.block, st);
  };
  if (E.dtype == DEC_BPM_C64)
    run(float{});
  else
    run(double{});
  decbpm::check_launch();
  ABI_CATCH
}

int dec_bpm_linear_step(dec_bpm_t h, void* field, double dz, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_pml(h->E, "dec_bpm_linear_step");
  Engine& E = h->E;
  decbpm::check_prop_args(E, field, dz, 1, 0.0);
  hipStream_t st = as_stream(stream);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const decbpm::DevOps<T> d = E.ops<T>();
    decbpm::launch_perm_in<T>(d, E.perm, field, E.psi, 0, E.block, st);
    decbpm::lin_step<T>(E, d, E.psi, E.psi, E.ya, E.yb, E.ya, dz, nullptr, 0.0, st);
    decbpm::launch_perm_out<T>(d, E.perm, E.psi, field, 0, E.flag, E.block, st);
  };
  if (E.dtype == DEC_BPM_C64)
    run(float{});
  else
    run(double{});
  decbpm::check_launch();
  ABI_CATCH
}

int dec_bpm_propagate(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream) {
  ABI_TRY
  need(h);
  decbpm::check_prop_args(h->E, field, dz, n_steps, gamma);
  decbpm::propagate(h->E, field, dz, n_steps, gamma, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_propagate_noalloc(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream) {
  ABI_TRY
  need(h);
  decbpm::check_prop_args(h->E, field, dz, n_steps, gamma);
  decbpm::check_noalloc(h->E);
  if (h->E.dtype == DEC_BPM_C64)
    decbpm::propagate_noalloc_t<float>(h->E, field, dz, n_steps, gamma, as_stream(stream));
  else
    decbpm::propagate_noalloc_t<double>(h->E, field, dz, n_steps, gamma, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_propagate_unsplit(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_general(h->E, "dec_bpm_propagate_unsplit");
  decbpm::check_prop_args(h->E, field, dz, n_steps, gamma);
  if (!h->E.has_step || h->E.F != 1)
    fail(DEC_BPM_EINVAL,
         "the unsplit integrator runs on the one-field step tiles: not available with the beta4 term or with rows of "
         "more than 12 neighbours");
  if (h->E.dtype == DEC_BPM_C64)
    decbpm::propagate_unsplit_t<float>(h->E, field, dz, n_steps, gamma, as_stream(stream));
  else
    decbpm::propagate_unsplit_t<double>(h->E, field, dz, n_steps, gamma, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_propagate_adaptive(dec_bpm_t h, void* field, double z_end, double h0, double gamma, double rtol,
                               double atol, int64_t max_attempts, int64_t* n_accepted, int64_t* n_rejected,
                               double* last_h, double* z_reached, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_general(h->E, "dec_bpm_propagate_adaptive");
  Engine& E = h->E;
  if (n_accepted) *n_accepted = 0;
  if (n_rejected) *n_rejected = 0;
  if (last_h) *last_h = 0.0;
  if (z_reached) *z_reached = 0.0;
  if (!field) fail(DEC_BPM_EINVAL, "field is NULL");
  if (!(z_end >= 0.0) || !std::isfinite(z_end)) fail(DEC_BPM_EINVAL, "z_end must be finite and >= 0");
  if (!(h0 > 0.0) || !std::isfinite(h0)) fail(DEC_BPM_EINVAL, "h0 must be finite and > 0");
  if (!(rtol >= 0.0) || !(atol > 0.0) || !std::isfinite(rtol) || !std::isfinite(atol))
    fail(DEC_BPM_EINVAL, "need rtol >= 0 and atol > 0");
  if (!std::isfinite(gamma)) fail(DEC_BPM_EINVAL, "gamma must be finite");
  if (max_attempts < 1) fail(DEC_BPM_EINVAL, "max_attempts must be >= 1");
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  if (!E.has_step || E.F != 1)
    fail(DEC_BPM_EINVAL,
         "the adaptive integrator runs on one-field step tiles: not available with the beta4 term or with rows of "
         "more than 12 neighbours");
  if (z_end == 0.0) return DEC_BPM_OK;
  const bool ok = E.dtype == DEC_BPM_C64 ? decbpm::ensure_dp5_tiles<float>(E) : decbpm::ensure_dp5_tiles<double>(E);
  if (!ok) fail(DEC_BPM_EINVAL, "no seven-ring tiling of this mesh fits the adaptive kernel's LDS budget");
  hipStream_t st = as_stream(stream);
  const decbpm::AdaptiveResult r =
      E.dtype == DEC_BPM_C64
          ? decbpm::propagate_adaptive_t<float>(E, field, z_end, h0, gamma, rtol, atol, max_attempts, st)
          : decbpm::propagate_adaptive_t<double>(E, field, z_end, h0, gamma, rtol, atol, max_attempts, st);
  if (n_accepted) *n_accepted = r.accepted;
  if (n_rejected) *n_rejected = r.rejected;
  if (last_h) *last_h = r.last_h;
  if (z_reached) *z_reached = r.z;
  if (r.status == 1) fail(DEC_BPM_EUNSTABLE, "adaptive run: max_attempts trials did not reach z_end");
  if (r.status == 2) fail(DEC_BPM_ENONFINITE, "adaptive run: non-finite error norm");
  if (r.status == 3) fail(DEC_BPM_EUNSTABLE, "adaptive run: step size fell below 10 ulp of z");
  ABI_CATCH
}

int dec_bpm_find_mode(dec_bpm_t h, void* field, double power, double dtau, double gamma, double tol,
                      int64_t max_iter, double* mu, double* residual, int64_t* iterations, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_general(h->E, "dec_bpm_find_mode");
  decbpm::no_pml(h->E, "dec_bpm_find_mode");
  Engine& E = h->E;
  if (mu) *mu = 0.0;
  if (residual) *residual = 0.0;
  if (iterations) *iterations = 0;
  if (!field) fail(DEC_BPM_EINVAL, "field is NULL");
  if (!(power > 0.0) || !std::isfinite(power)) fail(DEC_BPM_EINVAL, "power must be finite and > 0");
  if (!(dtau > 0.0) || !std::isfinite(dtau)) fail(DEC_BPM_EINVAL, "dtau must be finite and > 0");
  if (!(tol >= 0.0) || !std::isfinite(tol)) fail(DEC_BPM_EINVAL, "tol must be finite and >= 0");
  if (!std::isfinite(gamma)) fail(DEC_BPM_EINVAL, "gamma must be finite");
  if (max_iter < 1) fail(DEC_BPM_EINVAL, "max_iter must be >= 1");
  decbpm::check_stability(E, dtau);
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  if (!E.has_step || E.F != 1)
    fail(DEC_BPM_EINVAL,
         "the mode solver runs on one-field step tiles: not available with the beta4 term or with rows of more "
         "than 12 neighbours");
  hipStream_t st = as_stream(stream);
  const decbpm::ModeResult r =
      E.dtype == DEC_BPM_C64 ? decbpm::find_mode_t<float>(E, field, power, dtau, gamma, tol, max_iter, st)
                             : decbpm::find_mode_t<double>(E, field, power, dtau, gamma, tol, max_iter, st);
  if (mu) *mu = r.mu;
  if (residual) *residual = r.res;
  if (iterations) *iterations = r.iter;
  if (r.status == 1) fail(DEC_BPM_EUNSTABLE, "mode solver: no convergence within max_iter iterations");
  if (r.status == 2) fail(DEC_BPM_ENONFINITE, "mode solver: zero or non-finite power or quotient");
  ABI_CATCH
}

static void check_finite(Engine& E, void* stream) {
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  int f = 0;
  HIP_OK(hipMemcpyAsync(&f, E.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (f) {
    HIP_OK(hipMemsetAsync(E.flag, 0, sizeof(int), st));
    HIP_OK(hipStreamSynchronize(st));
    fail(DEC_BPM_ENONFINITE, (f & 2) ? "a persistent launch timed out waiting for a neighbour tile (its output is invalid)"
                                      : "a propagated field contains NaN or Inf");
  }
}

int dec_bpm_check_finite(dec_bpm_t h, void* stream) {
  ABI_TRY
  need(h);
  check_finite(h->E, stream);
  ABI_CATCH
}

int dec_bpm_batch_check_finite(dec_bpm_batch_t b, void* stream) {
  ABI_TRY
  if (!b) fail(DEC_BPM_EINVAL, "batch is NULL");
  check_finite(b->E, stream);
  ABI_CATCH
}

int dec_bpm_diagnostics(dec_bpm_t h, const void* field, double gamma, double* power, double* hamiltonian,
                        void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!field) fail(DEC_BPM_EINVAL, "field is NULL");
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const decbpm::DevOps<T> d = E.ops<T>();
    decbpm::launch_perm_in<T>(d, E.perm, field, E.ya, 0, E.block, st);
    decbpm::launch_diag<T>(d, E.ya, gamma, E.partials, E.n_red_blocks, E.red_out, st);
  };
  if (E.dtype == DEC_BPM_C64)
    run(float{});
  else
    run(double{});
  decbpm::check_launch();
  double out[2];
  HIP_OK(hipMemcpyAsync(out, E.red_out, sizeof out, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (power) *power = out[0];
  // with a PML the Hamiltonian is not defined (complex L): NaN
  if (hamiltonian) *hamiltonian = (E.pml || E.general()) ? std::nan("") : out[1];
  ABI_CATCH
}

int dec_bpm_overlap(dec_bpm_t h, const void* a, const void* b, double* re, double* im, void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!a || !b) fail(DEC_BPM_EINVAL, "a and b must not be NULL");
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  hipStream_t st = as_stream(stream);
  if (E.dtype == DEC_BPM_C64)
    decbpm::launch_overlap<float>(E.n_rows, E.h0c, a, b, E.partials, E.n_red_blocks, E.red_out, st);
  else
    decbpm::launch_overlap<double>(E.n_rows, E.h0c, a, b, E.partials, E.n_red_blocks, E.red_out, st);
  decbpm::check_launch();
  double out[2];
  HIP_OK(hipMemcpyAsync(out, E.red_out, sizeof out, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (re) *re = out[0];
  if (im) *im = out[1];
  ABI_CATCH
}

int dec_bpm_workspace_size(dec_bpm_t h, int64_t n_steps, int64_t every, size_t* bytes) {
  ABI_TRY
  need(h);
  if (!bytes || n_steps < 0 || every < 0) fail(DEC_BPM_EINVAL, "bad workspace query");
  *bytes = decbpm::ws_layout(h->E, n_steps, every).total;
  ABI_CATCH
}

int dec_bpm_forward_checkpointed(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, int64_t every,
                                 void* workspace, size_t ws_bytes, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_general(h->E, "dec_bpm_forward_checkpointed");
  Engine& E = h->E;
  decbpm::pml_adjoint_ok(E, "dec_bpm_forward_checkpointed");
  decbpm::check_prop_args(E, field, dz, n_steps, gamma);
  if (every < 0) fail(DEC_BPM_EINVAL, "every must be >= 0");
  const auto L = decbpm::ws_layout(E, n_steps, every);
  if (!workspace || ws_bytes < L.total)
    fail(DEC_BPM_EWORKSPACE, "workspace needs " + std::to_string(L.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) fail(DEC_BPM_EWORKSPACE, "workspace must be 256-byte aligned");
  char* ws = static_cast<char*>(workspace);
  const bool recorded = E.dtype == DEC_BPM_C64
                            ? decbpm::forward_ckpt_t<float>(E, field, dz, n_steps, gamma, every, ws, as_stream(stream))
                            : decbpm::forward_ckpt_t<double>(E, field, dz, n_steps, gamma, every, ws, as_stream(stream));
  Engine::CkptRec rec;
  rec.ws = workspace;
  rec.dz = dz;
  rec.gamma = gamma;
  rec.n = n_steps;
  rec.every = L.S;
  rec.dn_digest = E.dn_digest;
  rec.last_recorded = recorded;
  auto& cs = E.ckpts;
  cs.erase(std::remove_if(cs.begin(), cs.end(), [&](const Engine::CkptRec& c) { return c.ws == workspace; }),
           cs.end());
  if (cs.size() >= Engine::kMaxCkpt) cs.erase(cs.begin());
  cs.push_back(rec);
  ABI_CATCH
}

int dec_bpm_adjoint(dec_bpm_t h, const void* grad_out, double dz, int64_t n_steps, double gamma, int64_t every,
                    void* workspace, size_t ws_bytes, void* grad_field0, double* grad_dn, void* stream) {
  ABI_TRY
  need(h);
  decbpm::no_general(h->E, "dec_bpm_adjoint");
  Engine& E = h->E;
  decbpm::pml_adjoint_ok(E, "dec_bpm_adjoint");
  decbpm::check_prop_args(E, grad_field0, dz, n_steps, gamma);
  if (!grad_out) fail(DEC_BPM_EINVAL, "grad_out is NULL");
  const auto L = decbpm::ws_layout(E, n_steps, every);
  if (!workspace || ws_bytes < L.total)
    fail(DEC_BPM_EWORKSPACE, "workspace needs " + std::to_string(L.total) + " bytes");
  const auto rec = std::find_if(E.ckpts.begin(), E.ckpts.end(),
                                [&](const Engine::CkptRec& c) { return c.ws == workspace; });
  if (rec == E.ckpts.end() || rec->dz != dz || rec->gamma != gamma || rec->n != n_steps || rec->every != L.S ||
      rec->dn_digest != E.dn_digest)
    fail(DEC_BPM_EWORKSPACE, "workspace does not hold the checkpoints of a matching forward call");
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = as_stream(stream);
  const bool step = E.dtype == DEC_BPM_C64 ? decbpm::use_step_adjoint<float>(E) : decbpm::use_step_adjoint<double>(E);
  const bool recorded = step && rec->last_recorded;
  // a recompute overwrites the segment store: the last segment's record then no longer holds
  if (!(recorded && L.K == 1)) rec->last_recorded = false;
  if (E.dtype == DEC_BPM_C64) {
    if (step)
      decbpm::adjoint_step_t<float>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, recorded, st);
    else if (decbpm::adjoint_fused_ok<float>(E))
      decbpm::adjoint_fused_t<float>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, st);
    else
      decbpm::adjoint_t<float>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, st);
  } else {
    if (step)
      decbpm::adjoint_step_t<double>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, recorded, st);
    else if (decbpm::adjoint_fused_ok<double>(E))
      decbpm::adjoint_fused_t<double>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, st);
    else
      decbpm::adjoint_t<double>(E, grad_out, dz, n_steps, gamma, every, ws, grad_field0, grad_dn, st);
  }
  ABI_CATCH
}

int dec_bpm_batch_create(const dec_bpm_t* meshes, int32_t n_meshes, const int32_t* fields_per_mesh,
                         dec_bpm_batch_t* out) {
  ABI_TRY
  if (!out) fail(DEC_BPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!meshes || n_meshes < 1) fail(DEC_BPM_EINVAL, "need at least one mesh");
  if (!fields_per_mesh) fail(DEC_BPM_EINVAL, "fields_per_mesh is NULL");
  int32_t fmax = 0;
  for (int32_t m = 0; m < n_meshes; ++m) {
    if (fields_per_mesh[m] < 1 || fields_per_mesh[m] > 4096)
      fail(DEC_BPM_EINVAL, "every mesh needs between 1 and 4096 fields");
    fmax = std::max(fmax, fields_per_mesh[m]);
  }
  std::vector<const decbpm::Assembled*> list;
  std::vector<int> lumped;
  const dec_bpm_s* m0 = meshes[0];
  if (!m0) fail(DEC_BPM_EINVAL, "NULL mesh handle");
  double rho = 0;
  for (int32_t m = 0; m < n_meshes; ++m) {
    const dec_bpm_s* h = meshes[m];
    if (!h) fail(DEC_BPM_EINVAL, "NULL mesh handle");
    if (!h->A.kp_re.empty()) fail(DEC_BPM_EINVAL, "batches do not take meshes with a PML");
    if (h->E.general()) fail(DEC_BPM_EINVAL, "batches do not take L^3, L^4 or non-Kerr responses");
    if (h->opt.dtype != m0->opt.dtype || h->opt.p1 != m0->opt.p1 || h->opt.beta4 != m0->opt.beta4 ||
        h->opt.nonlinearity != m0->opt.nonlinearity || h->opt.host_only != m0->opt.host_only)
      fail(DEC_BPM_EINVAL, "all meshes of a batch must share dtype, p1, beta4, nonlinearity and host_only");
    list.push_back(&h->A);
    lumped.push_back(h->opt.nonlinearity == DEC_BPM_NL_LUMPED ? 1 : 0);
    rho = std::max(rho, h->A.rho);
  }
  std::unique_ptr<dec_bpm_batch_s> b(new dec_bpm_batch_s());
  Engine& E = b->E;
  E.dtype = m0->opt.dtype;
  // the device carries the largest field count on every row, rounded up to
  // whole groups of the batched tile kernels (32 bytes of fields per slot);
  // one field per mesh stays a one-field engine
  const int32_t vf = E.dtype == DEC_BPM_C64 ? 4 : 2;
  E.F = fmax == 1 ? 1 : (fmax + vf - 1) / vf * vf;
  E.fpm.assign(fields_per_mesh, fields_per_mesh + n_meshes);
  E.p1 = m0->opt.p1;
  E.beta4 = m0->opt.beta4;
  E.nl = m0->opt.nonlinearity;
  E.rho = rho;
  E.n_rows = 0;
  for (auto* a : list) E.n_rows += a->n;
  if (!m0->opt.host_only) decbpm::build_engine(E, list, lumped);  // host-only meshes: a host-only batch
  for (int32_t m = 0; m < n_meshes; ++m) b->n_elems += list[m]->n * fields_per_mesh[m];
  *out = b.release();
  ABI_CATCH
}

void dec_bpm_batch_destroy(dec_bpm_batch_t b) { delete b; }

int dec_bpm_batch_size(dec_bpm_batch_t b, int64_t* n_elems) {
  ABI_TRY
  if (!b || !n_elems) fail(DEC_BPM_EINVAL, "NULL argument");
  *n_elems = b->n_elems;
  ABI_CATCH
}

int dec_bpm_batch_propagate(dec_bpm_batch_t b, void* packed_fields, double dz, int64_t n_steps, double gamma,
                            void* stream) {
  ABI_TRY
  if (!b) fail(DEC_BPM_EINVAL, "batch is NULL");
  decbpm::check_prop_args(b->E, packed_fields, dz, n_steps, gamma);
  decbpm::propagate(b->E, packed_fields, dz, n_steps, gamma, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_autotune(dec_bpm_t h, double dz, double gamma, void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  decbpm::check_prop_args(E, E.psi, dz, 1, gamma);
  if (E.dtype == DEC_BPM_C64)
    decbpm::autotune_t<float>(E, dz, gamma, as_stream(stream));
  else
    decbpm::autotune_t<double>(E, dz, gamma, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_batch_autotune(dec_bpm_batch_t b, double dz, double gamma, void* stream) {
  ABI_TRY
  if (!b) fail(DEC_BPM_EINVAL, "batch is NULL");
  Engine& E = b->E;
  decbpm::check_prop_args(E, E.psi, dz, 1, gamma);
  if (E.dtype == DEC_BPM_C64)
    decbpm::autotune_t<float>(E, dz, gamma, as_stream(stream));
  else
    decbpm::autotune_t<double>(E, dz, gamma, as_stream(stream));
  ABI_CATCH
}

static void get_tuning(const Engine& E, dec_bpm_tuning* t) {
  t->block_size = E.block;
  t->steps_per_graph = E.spg;
  t->fused = (E.has_tiles || E.has_btiles || E.has_step || E.has_step4 || E.has_sfl) ? E.fused : 0;
  t->tile_block = E.has_tiles ? E.tblock() : E.tile_block;
  t->xcd_remap = E.xcd;
}

static void set_tuning(Engine& E, const dec_bpm_tuning* t) {
  if (!t || t->block_size < 64 || t->block_size > 1024 || t->block_size % 64 || t->steps_per_graph < 1 ||
      t->tile_block < 64 || t->tile_block > 1024 || t->tile_block % 64 || (t->fused < 0 || t->fused > 3) ||
      (t->xcd_remap != 0 && t->xcd_remap != 1))
    fail(DEC_BPM_EINVAL, "bad tuning");
  if (E.pml && t->fused != 2 && t->fused != 3)
    fail(DEC_BPM_EINVAL, "a PML handle runs the one-kernel step or the persistent launch only (fused = 2 or 3)");
  if (E.high_order() && t->fused != 0)
    fail(DEC_BPM_EINVAL, "L^3 and L^4 terms run the five-kernel path only (fused = 0)");
  E.block = t->block_size;
  E.spg = t->steps_per_graph;
  E.fused = t->fused;
  E.tile_block = t->tile_block;
  E.xcd = t->xcd_remap;
}

int dec_bpm_batch_get_tuning(dec_bpm_batch_t b, dec_bpm_tuning* t) {
  ABI_TRY
  if (!b || !t) fail(DEC_BPM_EINVAL, "NULL argument");
  get_tuning(b->E, t);
  ABI_CATCH
}

int dec_bpm_batch_set_tuning(dec_bpm_batch_t b, const dec_bpm_tuning* t) {
  ABI_TRY
  if (!b) fail(DEC_BPM_EINVAL, "batch is NULL");
  set_tuning(b->E, t);
  ABI_CATCH
}

int dec_bpm_get_tuning(dec_bpm_t h, dec_bpm_tuning* t) {
  ABI_TRY
  need(h);
  if (!t) fail(DEC_BPM_EINVAL, "NULL tuning");
  get_tuning(h->E, t);
  ABI_CATCH
}

int dec_bpm_set_tuning(dec_bpm_t h, const dec_bpm_tuning* t) {
  ABI_TRY
  need(h);
  set_tuning(h->E, t);
  ABI_CATCH
}

int dec_bpm_time_kernels(dec_bpm_t h, double dz, double gamma, int32_t reps, double* ms, double* bytes,
                         void* stream) {
  ABI_TRY
  need(h);
  Engine& E = h->E;
  if (!E.on_device) fail(DEC_BPM_ENODEVICE, "handle was created host-only");
  decbpm::check_prop_args(E, E.psi, dz, 1, gamma);
  if (reps < 1) fail(DEC_BPM_EINVAL, "reps must be >= 1");
  if (E.dtype == DEC_BPM_C64)
    decbpm::time_kernels_t<float>(E, dz, gamma, reps, ms, bytes, as_stream(stream));
  else
    decbpm::time_kernels_t<double>(E, dz, gamma, reps, ms, bytes, as_stream(stream));
  ABI_CATCH
}

int dec_bpm_batch_time_kernels(dec_bpm_batch_t b, double dz, double gamma, int32_t reps, double* ms, double* bytes,
                               void* stream) {
  ABI_TRY
  if (!b) fail(DEC_BPM_EINVAL, "batch is NULL");
  Engine& E = b->E;
  decbpm::check_prop_args(E, E.psi, dz, 1, gamma);
  if (reps < 1) fail(DEC_BPM_EINVAL, "reps must be >= 1");
  if (E.dtype == DEC_BPM_C64)
    decbpm::time_kernels_t<float>(E, dz, gamma, reps, ms, bytes, as_stream(stream));
  else
    decbpm::time_kernels_t<double>(E, dz, gamma, reps, ms, bytes, as_stream(stream));
  ABI_CATCH
}

}  // extern "C"
