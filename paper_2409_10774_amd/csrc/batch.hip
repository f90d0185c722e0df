// Resident batches of RVEs and the request-serving loops built on them
// (C ABI in include/mp.h: mp_batch_*, mp_serve_*).
//
// A batch owns a caller-provided device arena.  Each admitted RVE takes one
// region of it (spectra, fields, history, phase map, constants, twiddles,
// load path, step records) and one descriptor slot; its whole load path then
// runs on the device (batch.hpp).  mp_batch_run replays a graph of
// iters_per_launch loop iterations of every resident RVE and reads back the
// slot states; finished RVEs stay readable until released, which returns
// their region to the arena.
#include "batch.hpp"
#include "host.hpp"

#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

using namespace mp;

namespace {

// First-fit allocator over [0, bytes) of the arena, 256-byte granules,
// neighbours coalesced on release.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// y / z pass schedule of a shape class: tile width and persistent grid
struct PassSched {
  int tx, grid;
  float ms;   // autotuner's time per launch (0: not tuned)
};

struct ClassInfo {
  int n[3];
  Geometry g;
  PassSched pass[3];   // Y_FWD, Z_GREEN, Y_INV
  int xgrid;
  bool an;             // an RVE with Eq. 5 phases or a tensor reference was admitted:
                       // the x pass's Eq. 5 variant
  bool tensor;         // an RVE with a tensor reference medium or a stored Green
                       // operator was admitted: Z_GREEN_AN (its solve per tile)
  bool al;             // an augmented-Lagrangian RVE was admitted: the ITER x pass
                       // that runs each RVE's own scheme
};

struct RveHost {
  int slot, cls, n_steps;
  size_t off, bytes;
  Layout L;
  size_t path_off, rec_off;
  long nvox;
};

// bytes of an RVE's region: the plan layout, its load path and step records
size_t rve_bytes(const Layout& L, int n_steps, size_t* path_off, size_t* rec_off) {
  size_t o = L.total;
  *path_off = o;
  o += align256(size_t(n_steps + 1 + 18 * n_steps) * sizeof(double));
  *rec_off = o;
  o += align256(size_t(n_steps) * kRec * sizeof(double));
  return o;
}

constexpr int kPassMode[3] = {Y_FWD, Z_GREEN, Y_INV};

}  // namespace

struct mp_batch_s {
  mp_batch_config cfg;
  size_t w;               // bytes per bulk word
  hipStream_t stream;     // caller's stream: every launch and copy
  hipStream_t cap;        // private stream used only to capture the graph
  unsigned char* ws;
  size_t bytes;
  Arena arena;
  void* rv;               // Rve<T>[kMaxSlots]
  Lists* ls;
  Lists* ls_host;         // pinned
  Lists* ls_ahead;        // pinned, the list header only: drain's second read-back
  hipEvent_t drained[2];  // drain: read-back of launch k done (k even, k odd)
  size_t base_bytes;      // descriptors + lists at the head of the arena
  std::vector<ClassInfo> cls;
  std::vector<int> slot_id;   // id held by each slot, -1 = free
  std::map<int, RveHost> rves;
  int next_id;
  int cus;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
  long graph_launches;
};

namespace {

// ---------------------------------------------------------------------------
// compile-time size dispatch of the batch kernels
// ---------------------------------------------------------------------------
constexpr int tx_half(int L) { return tx_wide(L) > 1 ? tx_wide(L) / 2 : 1; }

template <class T, int MODE, int L, int TX>
const void* axis_fn() {
  return reinterpret_cast<const void*>(&k_batch_axis<T, MODE, L, TX>);
}

// kernel, threads and LDS bytes of the batch axis pass (MODE, L, tx);
// tx must be 1, tx_half(L) or tx_wide(L)
template <class T, int MODE>
bool axis_kernel(int L, int tx, const void** fn, int* nthr, size_t* shm) {
  switch (L) {
#define MP_CASE(N)                                                                  \
  case N:                                                                           \
    if (tx == 1) {                                                                  \
      *fn = axis_fn<T, MODE, N, 1>();                                               \
      *nthr = AShape<N, 1>::NTHR;                                                   \
      *shm = AShape<N, 1>::LDS * sizeof(cx<T>);                                     \
    } else if (tx == tx_half(N)) {                                                  \
      *fn = axis_fn<T, MODE, N, tx_half(N)>();                                      \
      *nthr = AShape<N, tx_half(N)>::NTHR;                                          \
      *shm = AShape<N, tx_half(N)>::LDS * sizeof(cx<T>);                            \
    } else if (tx == tx_wide(N)) {                                                  \
      *fn = axis_fn<T, MODE, N, tx_wide(N)>();                                      \
      *nthr = AShape<N, tx_wide(N)>::NTHR;                                          \
      *shm = AShape<N, tx_wide(N)>::LDS * sizeof(cx<T>);                            \
    } else {                                                                        \
      return false;                                                                 \
    }                                                                               \
    return true;
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
  return false;
}

template <class T, int MODE>
bool x_kernel(int n0, bool an, bool al, const void** fn, int* nthr) {
  switch (n0) {
#define MP_CASE(N)                                                                            \
  case N:                                                                                     \
    *fn = an ? reinterpret_cast<const void*>(&k_batch_x<T, MODE, N, true>)                    \
             : reinterpret_cast<const void*>(&k_batch_x<T, MODE, N, false>);                  \
    if constexpr (sizeof(T) == sizeof(double) && MODE == X_ITER) {                            \
      if (al)                                                                                 \
        *fn = an ? reinterpret_cast<const void*>(&k_batch_x<T, MODE, N, true, true>)          \
                 : reinterpret_cast<const void*>(&k_batch_x<T, MODE, N, false, true>);        \
    }                                                                                         \
    *nthr = XShape<T, N>::NTHR;                                                               \
    return true;
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
  return false;
}

// launch through the generic entry (the kernel is selected above)
hipError_t launch(const void* fn, int grid, int nthr, size_t shm, hipStream_t s, void** args) {
  return hipLaunchKernel(fn, dim3(grid), dim3(nthr), args, shm, s);
}

template <class T>
struct BEng {
  static Rve<T>* rv(mp_batch B) { return static_cast<Rve<T>*>(B->rv); }

  static hipError_t axis(mp_batch B, int c, int p, const Rve<T>* rvp, const Lists* lsp, int tx,
                         int grid, hipStream_t s) {
    const ClassInfo& C = B->cls[c];
    const void* fn;
    int nthr;
    size_t shm;
    const int mode = kPassMode[p];
    const int L = mode == Z_GREEN ? C.n[2] : C.n[1];
    bool ok = mode == Y_FWD   ? axis_kernel<T, Y_FWD>(L, tx, &fn, &nthr, &shm)
              : mode == Y_INV ? axis_kernel<T, Y_INV>(L, tx, &fn, &nthr, &shm)
              : C.tensor      ? axis_kernel<T, Z_GREEN_AN>(L, tx, &fn, &nthr, &shm)
                              : axis_kernel<T, Z_GREEN>(L, tx, &fn, &nthr, &shm);
    if (!ok) return hipErrorInvalidValue;
    int cls = c, gx = C.g.nh / tx, gy = mode == Z_GREEN ? C.n[1] : C.n[2];
    void* args[] = {&rvp, &lsp, &cls, &gx, &gy};
    return launch(fn, grid, nthr, shm, s, args);
  }

  static hipError_t xpass(mp_batch B, int c, int mode, hipStream_t s) {
    const ClassInfo& C = B->cls[c];
    const void* fn;
    int nthr;
    if (!(mode == X_ITER ? x_kernel<T, X_ITER>(C.n[0], C.an, C.al, &fn, &nthr)
                         : x_kernel<T, X_TRANS>(C.n[0], C.an, false, &fn, &nthr)))
      return hipErrorInvalidValue;
    const Rve<T>* rvp = rv(B);
    const Lists* lsp = B->ls;
    int cls = c, tiles = C.g.xblocks;
    void* args[] = {&rvp, &lsp, &cls, &tiles};
    // transitions alone are rare (once per step of an RVE): a grid that
    // fills the chip about once, so that an iteration without any costs
    // little; a multiple of 16: the two levels of an item then share an XCD
    // (x_item)
    const int grid = ((mode == X_ITER ? C.xgrid : std::min(C.xgrid, 4 * B->cus)) + 15) / 16 * 16;
    return launch(fn, grid, nthr, 0, s, args);
  }

  static hipError_t ctl(mp_batch B, int update, hipStream_t s) {
    hipLaunchKernelGGL((k_batch_ctl<T>), dim3(1), dim3(kMaxSlots), 0, s, rv(B), B->ls,
                       int(B->cls.size()), update);
    return hipGetLastError();
  }

  // one loop iteration of every resident RVE
  static hipError_t iteration(mp_batch B, hipStream_t s) {
    hipError_t e;
    for (int c = 0; c < int(B->cls.size()); ++c)
      for (int p = 0; p < 3; ++p)
        if ((e = axis(B, c, p, rv(B), B->ls, B->cls[c].pass[p].tx, B->cls[c].pass[p].grid, s)) !=
            hipSuccess)
          return e;
    // loop iterations, then step transitions (in low precision the ITER
    // kernel takes both)
    for (int c = 0; c < int(B->cls.size()); ++c) {
      if ((e = xpass(B, c, X_ITER, s)) != hipSuccess) return e;
      if (!x_merged<T>() && (e = xpass(B, c, X_TRANS, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batch_rows<T>), dim3(4 * B->cus), dim3(256), 0, s, rv(B), B->ls,
                       int(B->cls.size()));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return ctl(B, 1, s);
  }

  // Grid of a pass: 8 times the blocks the CUs have wave slots for (32
  // waves per CU).  Blocks stride over the work items; extra blocks find no
  // item and exit.  The grid does not depend on an occupancy estimate.
  static hipError_t occupancy(const void* fn, int nthr, size_t shm, int cus, int* grid) {
    (void)fn;
    (void)shm;
    const int waves = (nthr + 63) / 64;
    *grid = 8 * cus * std::max(1, 32 / waves);
    return hipSuccess;
  }

  static hipError_t allow_all() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
      const int sizes[] = {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
      for (int L : sizes) {
        int cand[3];
        int nc = 0;
        // 1, tx_half(L), tx_wide(L)
        int tw = 1;
        while (2 * tw * L <= 256) tw *= 2;
        cand[nc++] = 1;
        cand[nc++] = tw > 1 ? tw / 2 : 1;
        cand[nc++] = tw;
        for (int k = 0; k < nc; ++k)
          for (int p = 0; p < 4; ++p) {
            const void* fn;
            int nthr;
            size_t shm;
            bool ok = p == 0   ? axis_kernel<T, Y_FWD>(L, cand[k], &fn, &nthr, &shm)
                      : p == 2 ? axis_kernel<T, Y_INV>(L, cand[k], &fn, &nthr, &shm)
                      : p == 3 ? axis_kernel<T, Z_GREEN_AN>(L, cand[k], &fn, &nthr, &shm)
                               : axis_kernel<T, Z_GREEN>(L, cand[k], &fn, &nthr, &shm);
            if (!ok) continue;
            hipError_t e =
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
            if (e != hipSuccess && err == hipSuccess) err = e;
          }
      }
    });
    return err;
  }

  static mp_status setup_class(mp_batch B, ClassInfo& C);
  static mp_status admit(mp_batch B, const mp_problem* prob, int32_t n_steps, const double* times,
                         const double* E, const double* Gam, int32_t* id);
};

// default schedule of a class: the single-RVE tile widths, full occupancy
template <class T>
mp_status default_sched(mp_batch B, ClassInfo& C) {
  const Geometry& g = C.g;
  for (int p = 0; p < 3; ++p) {
    const int mode = kPassMode[p];
    const int tx = mode == Z_GREEN ? g.txz : g.txy;
    const int L = mode == Z_GREEN ? C.n[2] : C.n[1];
    const void* fn;
    int nthr;
    size_t shm;
    bool ok = mode == Y_FWD   ? axis_kernel<T, Y_FWD>(L, tx, &fn, &nthr, &shm)
              : mode == Y_INV ? axis_kernel<T, Y_INV>(L, tx, &fn, &nthr, &shm)
                              : axis_kernel<T, Z_GREEN>(L, tx, &fn, &nthr, &shm);
    if (!ok) return fail(MP_E_INVALID, "no kernel for axis length " + std::to_string(L));
    int grid;
    HIP_TRY(BEng<T>::occupancy(fn, nthr, shm, B->cus, &grid));
    C.pass[p] = PassSched{tx, grid, 0.f};
  }
  const void* fn;
  int nthr;
  if (!x_kernel<T, X_ITER>(C.n[0], C.an, false, &fn, &nthr)) return fail(MP_E_INVALID, "no x kernel");
  HIP_TRY(BEng<T>::occupancy(fn, nthr, 0, B->cus, &C.xgrid));
  return MP_OK;
}

// Autotuner: for each y / z pass of a class, time every tile width in
// {1, wide / 2, wide} (wide = the largest with TX * L <= 256 dividing n0/2)
// with the full persistent grid, a quarter of it and the blocks the chip
// holds at once, on replicas of the class's spectrum (enough replicas for
// about 2^23 voxels), keep the fastest.  Results are cached per (precision,
// shape) for the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::array<PassSched, 3>> g_tune_cache;

template <class T>
mp_status BEng<T>::setup_class(mp_batch B, ClassInfo& C) {
  mp_status st = default_sched<T>(B, C);
  if (st != MP_OK || !B->cfg.autotune) return st;
  const auto key = std::make_tuple(int(sizeof(T)), C.n[0], C.n[1], C.n[2]);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int p = 0; p < 3; ++p) C.pass[p] = it->second[p];
      return MP_OK;
    }
  }
  const Geometry& g = C.g;
  const size_t spec_bytes = align256(size_t(18) * g.nspec * sizeof(cx<T>));
  int reps = int(std::max<long>(1, (1L << 23) / g.nvox));
  reps = std::min(reps, kMaxSlots);
  // temporary region: reps spectra (zero), twiddles, descriptors, a list
  const size_t tw_bytes = align256(size_t(g.n0 + g.n1 + g.n2) * sizeof(cx<T>));
  size_t rv_bytes, need, off;
  for (;;) {   // as many replicas as the free arena allows (none: keep the defaults)
    rv_bytes = align256(size_t(reps) * sizeof(Rve<T>));
    need = size_t(reps) * spec_bytes + tw_bytes + rv_bytes + align256(sizeof(Lists));
    if (B->arena.alloc(need, &off)) break;
    if (reps == 1) return MP_OK;
    reps /= 2;
  }
  unsigned char* base = B->ws + off;
  auto cleanup = [&]() { B->arena.release(off, need); };
  std::vector<cx<T>> tw;
  twiddles(g.n0, &tw);
  twiddles(g.n1, &tw);
  twiddles(g.n2, &tw);
  cx<T>* twd = reinterpret_cast<cx<T>*>(base + size_t(reps) * spec_bytes);
  Rve<T>* trv = reinterpret_cast<Rve<T>*>(base + size_t(reps) * spec_bytes + tw_bytes);
  Lists* tls = reinterpret_cast<Lists*>(base + size_t(reps) * spec_bytes + tw_bytes + rv_bytes);
  std::vector<Rve<T>> hr(reps);
  std::vector<Lists> hl(1);
  std::memset(hr.data(), 0, hr.size() * sizeof(Rve<T>));
  std::memset(hl.data(), 0, sizeof(Lists));
  for (int r = 0; r < reps; ++r) {
    cx<T>* S = reinterpret_cast<cx<T>*>(base + size_t(r) * spec_bytes);
    AxisArgs<T>& y = hr[r].y;
    y.S = S;
    y.ostride = long(g.n1) * g.nh * 18;
    y.pstride = long(g.nh) * 18;
    y.tw = twd + g.n0;
    AxisArgs<T>& z = hr[r].z;
    z.S = S;
    z.ostride = long(g.nh) * 18;
    z.pstride = long(g.n1) * g.nh * 18;
    z.tw = twd + g.n0 + g.n1;
    z.n0 = g.n0;
    z.n1 = g.n1;
    z.n2 = g.n2;
    z.h = 1.0;
    z.scale = 1.0 / double(g.nvox);
    z.ref = RefC{1.0, 1.0, 0.5, 0.0, 1.0, 1.0};
  }
  const int ci = int(&C - B->cls.data());
  hl[0].ns[ci] = reps;
  for (int r = 0; r < reps; ++r) hl[0].s[ci][r] = r;
  std::vector<hipEvent_t> ev(2, nullptr);
  auto run = [&]() -> mp_status {
    HIP_TRY(hipMemsetAsync(base, 0, size_t(reps) * spec_bytes, B->stream));
    HIP_TRY(hipMemcpyAsync(twd, tw.data(), tw.size() * sizeof(cx<T>), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(trv, hr.data(), hr.size() * sizeof(Rve<T>), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(tls, hl.data(), sizeof(Lists), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    for (int p = 0; p < 3; ++p) {
      const int mode = kPassMode[p];
      const int L = mode == Z_GREEN ? g.n2 : g.n1;
      int tw_max = 1;
      while (2 * tw_max * L <= 256) tw_max *= 2;
      const int cands[3] = {1, tw_max > 1 ? tw_max / 2 : 1, tw_max};
      PassSched best = C.pass[p];
      float best_ms = 1e30f;
      for (int k = 0; k < 3; ++k) {
        const int tx = cands[k];
        if (k > 0 && tx == cands[k - 1]) continue;
        if (g.nh % tx) continue;
        const void* fn;
        int nthr;
        size_t shm;
        bool ok = mode == Y_FWD   ? axis_kernel<T, Y_FWD>(L, tx, &fn, &nthr, &shm)
                  : mode == Y_INV ? axis_kernel<T, Y_INV>(L, tx, &fn, &nthr, &shm)
                                  : axis_kernel<T, Z_GREEN>(L, tx, &fn, &nthr, &shm);
        if (!ok) continue;
        int full, per_cu = 0;
        HIP_TRY(occupancy(fn, nthr, shm, B->cus, &full));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nthr, shm));
        // the full grid, a quarter of it, and the blocks the chip holds at once
        const int grids[3] = {full, std::max(B->cus, full / 4), std::max(1, per_cu) * B->cus};
        for (int gi = 0; gi < 3; ++gi) {
          const int grid = grids[gi];
          if ((gi > 0 && grid == grids[0]) || (gi > 1 && grid == grids[1])) continue;
          HIP_TRY(axis(B, ci, p, trv, tls, tx, grid, B->stream));   // warm-up
          float ms = 0.f;
          for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipEventRecord(ev[0], B->stream));
            HIP_TRY(axis(B, ci, p, trv, tls, tx, grid, B->stream));
            HIP_TRY(hipEventRecord(ev[1], B->stream));
            HIP_TRY(hipEventSynchronize(ev[1]));
            float one = 0.f;
            HIP_TRY(hipEventElapsedTime(&one, ev[0], ev[1]));
            ms += one;
          }
          ms /= 3.f;
          if (ms < best_ms) {
            best_ms = ms;
            best = PassSched{tx, grid, ms / float(reps)};
          }
        }
      }
      C.pass[p] = best;
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MP_OK;
  };
  st = run();
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  cleanup();
  if (st != MP_OK) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = {C.pass[0], C.pass[1], C.pass[2]};
  return MP_OK;
}

template <class T>
mp_status BEng<T>::admit(mp_batch B, const mp_problem* prob, int32_t n_steps, const double* times,
                         const double* E, const double* Gam, int32_t* id) {
  Geometry g;
  mp_status st = validate(prob, &g);
  if (st != MP_OK) return st;
  int ci = -1;
  for (int c = 0; c < int(B->cls.size()); ++c)
    if (B->cls[c].n[0] == g.n0 && B->cls[c].n[1] == g.n1 && B->cls[c].n[2] == g.n2) ci = c;
  if (ci < 0) return fail(MP_E_INVALID, "grid shape is not one of the batch's shape classes");
  int slot = -1;
  for (int s = 0; s < B->cfg.max_rves; ++s)
    if (B->slot_id[s] < 0) {
      slot = s;
      break;
    }
  if (slot < 0) return fail(MP_E_NOMEM, "every slot of the batch is in use");
  RefC ref;
  if ((st = reference_medium(prob, g.nvox, &ref)) != MP_OK) return st;
  RveHost H{};
  H.L = layout(g, B->w);
  H.bytes = rve_bytes(H.L, n_steps, &H.path_off, &H.rec_off);
  if (!B->arena.alloc(H.bytes, &H.off)) return fail(MP_E_NOMEM, "the RVE does not fit in the free arena");
  H.slot = slot;
  H.cls = ci;
  H.n_steps = n_steps;
  H.nvox = g.nvox;
  unsigned char* b = B->ws + H.off;
  const Layout& L = H.L;

  std::vector<PhaseC> pc(256);
  for (int i = 0; i < prob->n_phases; ++i) pc[i] = derive(prob->phases[i]);
  std::vector<double> arows(aniso_words(g), 0.0);
  for (int j = 0; j < g.n_aniso; ++j) {
    aniso_rows(prob->aniso[j], &arows[size_t(j) * 162]);
    pc[prob->aniso[j].phase].t.aid = double(j);
  }
  if (g.ref_tensor) {
    // tensor reference medium: rows after the phases' records, then the
    // coefficients of its Fourier symbol (the plan's layout)
    mp_aniso r;
    if ((st = reference_tensors(prob, g.nvox, &r)) != MP_OK) {
      B->arena.release(H.off, H.bytes);
      return st;
    }
    aniso_rows(r, &arows[size_t(g.n_aniso) * 162]);
    green_symbol(r, &arows[sym_offset(g)]);
  } else if (g.green_stored) {
    // the symbol of the isotropic reference, from its Eq. 6 tensors, for
    // the stored Green operator
    mp_phase c{};
    c.lambda = ref.lam; c.mu = ref.mu; c.kappa = ref.kap;
    c.alpha = ref.alp; c.beta = ref.bet; c.gamma = ref.gam;
    mp_aniso r{};
    iso_tensors(c, r.A, r.B);
    green_symbol(r, &arows[sym_offset(g)]);
  }
  std::vector<cx<T>> tw;
  twiddles(g.n0, &tw);
  twiddles(g.n1, &tw);
  twiddles(g.n2, &tw);
  std::vector<double> path(size_t(n_steps + 1 + 18 * n_steps));
  std::copy(times, times + n_steps + 1, path.begin());
  std::copy(E, E + 9 * n_steps, path.begin() + n_steps + 1);
  std::copy(Gam, Gam + 9 * n_steps, path.begin() + n_steps + 1 + 9 * n_steps);

  Rve<T> R;
  std::memset(&R, 0, sizeof R);
  XArgs<T>& x = R.x;
  x.nrows = g.nrows;
  x.tw = reinterpret_cast<const cx<T>*>(b + L.tw);
  x.S = reinterpret_cast<cx<T>*>(b + L.S);
  x.nvox = g.nvox;
  x.E = reinterpret_cast<double*>(b + L.E);
  x.Eprev = reinterpret_cast<double*>(b + L.Eprev);
  x.base = reinterpret_cast<T*>(b + L.base);
  x.pq = reinterpret_cast<double*>(b + L.pq);
  x.out_tm = reinterpret_cast<T*>(b + L.out_tm);
  x.out_pq = reinterpret_cast<double*>(b + L.out_pq);
  x.phase = b + L.phase;
  x.params = reinterpret_cast<const PhaseC*>(b + L.params);
  x.partials = reinterpret_cast<double*>(b + L.partials);
  x.aniso = reinterpret_cast<const double*>(b + L.aniso);
  x.n_aniso = g.n_aniso;
  if (g.ref_tensor) x.refan = x.aniso + size_t(g.n_aniso) * 162;
  x.ref = ref;
  x.al = prob->scheme == MP_SCHEME_AL ? 1 : 0;
  x.relax = x.al ? prob->relax : 1.0;
  for (int c = 0; c < 9; ++c) {
    x.mac[c] = E[c];
    x.mac[9 + c] = Gam[c];
  }
  x.r = 0.0;
  x.first = 1;
  x.commit = 0;
  x.init = 1;
  AxisArgs<T>& y = R.y;
  y.S = x.S;
  y.ostride = long(g.n1) * g.nh * 18;
  y.pstride = long(g.nh) * 18;
  y.tw = x.tw + g.n0;
  AxisArgs<T>& z = R.z;
  z.S = x.S;
  z.ostride = long(g.nh) * 18;
  z.pstride = long(g.n1) * g.nh * 18;
  z.tw = x.tw + g.n0 + g.n1;
  z.n0 = g.n0;
  z.n1 = g.n1;
  z.n2 = g.n2;
  z.h = prob->h;
  z.scale = 1.0 / double(g.nvox);
  z.ref = ref;
  if (g.ref_tensor) z.gsym = x.aniso + sym_offset(g);
  if (g.green_stored) z.gtab = reinterpret_cast<const T*>(b + L.gtab);
  const double* pth = reinterpret_cast<const double*>(b + H.path_off);
  R.times = pth;
  R.Ep = pth + n_steps + 1;
  R.Gp = pth + n_steps + 1 + 9 * n_steps;
  R.rec = reinterpret_cast<double*>(b + H.rec_off);
  R.tol = prob->tol;
  R.nvox = g.nvox;
  R.xblocks = g.xblocks;
  R.state = RV_TRANS;
  R.cls = ci;
  R.step = 0;
  R.n_steps = n_steps;
  R.fixed = 0;
  R.max_iter = prob->max_iter;
  R.norm = prob->err_norm;

  auto undo = [&](mp_status s) {
    B->arena.release(H.off, H.bytes);
    return s;
  };
#define ADMIT_TRY(call)                                                         \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      g_err = std::string(#call) + ": " + hipGetErrorString(e_);                \
      return undo(MP_E_DEVICE);                                                 \
    }                                                                           \
  } while (0)
  ADMIT_TRY(hipMemsetAsync(b, 0, H.bytes, B->stream));
  ADMIT_TRY(hipMemcpyAsync(b + L.phase, prob->phase, g.nvox, hipMemcpyHostToDevice, B->stream));
  ADMIT_TRY(hipMemcpyAsync(b + L.params, pc.data(), pc.size() * sizeof(PhaseC), hipMemcpyHostToDevice,
                           B->stream));
  ADMIT_TRY(hipMemcpyAsync(b + L.aniso, arows.data(), arows.size() * sizeof(double), hipMemcpyHostToDevice,
                           B->stream));
  ADMIT_TRY(hipMemcpyAsync(b + L.tw, tw.data(), tw.size() * sizeof(cx<T>), hipMemcpyHostToDevice,
                           B->stream));
  ADMIT_TRY(hipMemcpyAsync(b + H.path_off, path.data(), path.size() * sizeof(double),
                           hipMemcpyHostToDevice, B->stream));
  if (g.green_stored) {
    // the stored Green operator (Sec. 2.4), once, from the symbol coefficients
    const int blocks = int(std::min<long>((g.nspec + 255) / 256, 4096));
    hipLaunchKernelGGL(k_green_table<T>, dim3(blocks), dim3(256), 0, B->stream,
                       x.aniso + sym_offset(g), g.n0, g.n1, g.n2, prob->h, reinterpret_cast<T*>(b + L.gtab));
    ADMIT_TRY(hipGetLastError());
  }
  ADMIT_TRY(hipMemcpyAsync(rv(B) + slot, &R, sizeof R, hipMemcpyHostToDevice, B->stream));
  ADMIT_TRY(ctl(B, 0, B->stream));
  // host arrays above are pageable and local: finish the copies here
  ADMIT_TRY(hipStreamSynchronize(B->stream));
#undef ADMIT_TRY
  *id = B->next_id++;
  B->slot_id[slot] = *id;
  B->rves[*id] = H;
  const bool an = g.n_aniso > 0 || g.ref_tensor;
  const bool tensor = g.ref_tensor || g.green_stored;
  const bool al = prob->scheme == MP_SCHEME_AL;
  if ((an && !B->cls[ci].an) || (tensor && !B->cls[ci].tensor) || (al && !B->cls[ci].al)) {
    // the class's x passes switch to the Eq. 5 variant, its z pass to the
    // general Green step: the next run captures the graph again (the stream
    // is idle, see above)
    B->cls[ci].an = B->cls[ci].an || an;
    B->cls[ci].tensor = B->cls[ci].tensor || tensor;
    B->cls[ci].al = B->cls[ci].al || al;
    if (B->captured) {
      (void)hipGraphExecDestroy(B->exec);
      (void)hipGraphDestroy(B->graph);
      B->exec = nullptr;
      B->graph = nullptr;
      B->captured = false;
    }
  }
  return MP_OK;
}

mp_status find(mp_batch B, int32_t id, RveHost** H) {
  if (!B) return fail(MP_E_INVALID, "batch is NULL");
  auto it = B->rves.find(id);
  if (it == B->rves.end()) return fail(MP_E_INVALID, "unknown RVE id " + std::to_string(id));
  *H = &it->second;
  return MP_OK;
}

// small fields of a descriptor (state, status, steps, iterations)
template <class T>
mp_status read_desc(mp_batch B, const RveHost& H, int* state, int* status, int* committed,
                    long* iters_total) {
  Rve<T> R;
  HIP_TRY(hipMemcpyAsync(&R, static_cast<Rve<T>*>(B->rv) + H.slot, sizeof R, hipMemcpyDeviceToHost,
                         B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  *state = R.state;
  *status = R.status;
  *committed = R.committed;
  *iters_total = R.iters_total;
  return MP_OK;
}

mp_status query(mp_batch B, const RveHost& H, int* state, int* status, int* committed, long* iters) {
  return B->w == sizeof(float) ? read_desc<float>(B, H, state, status, committed, iters)
                               : read_desc<double>(B, H, state, status, committed, iters);
}

// The records of RVE H's committed steps as mp_batch_response gives them
// (averages, error measure, iterations), rows past the committed ones NaN.
mp_status read_records(mp_batch B, const RveHost& H, int committed, double* out) {
  const size_t bytes = size_t(H.n_steps) * kRec * sizeof(double);
  HIP_TRY(hipMemcpyAsync(out, B->ws + H.off + H.rec_off, bytes, hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (int s = 0; s < H.n_steps; ++s) {
    double* r = out + size_t(s) * kRec;
    if (s >= committed) {
      for (int j = 0; j < kRec; ++j) r[j] = std::nan("");
      continue;
    }
    for (int j = 0; j < kNAvg; ++j) r[j] /= double(H.nvox);
  }
  return MP_OK;
}

int status_code(int s) {
  return s == RVS_NOT_CONVERGED ? MP_E_NOT_CONVERGED : s == RVS_DIVERGED ? MP_E_DIVERGED : MP_OK;
}

mp_status capture(mp_batch B) {
  if (B->captured) return MP_OK;
  hipError_t e;
  HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < B->cfg.iters_per_launch; ++k) {
    e = B->w == sizeof(float) ? BEng<float>::iteration(B, B->cap) : BEng<double>::iteration(B, B->cap);
    if (e != hipSuccess) {
      hipGraph_t junk;
      (void)hipStreamEndCapture(B->cap, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      return fail(MP_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
  }
  HIP_TRY(hipStreamEndCapture(B->cap, &B->graph));
  HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  B->captured = true;
  return MP_OK;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

mp_status mp_batch_footprint(const mp_batch_config* cfg, const mp_problem* prob, int32_t n_steps,
                             size_t* bytes) {
  if (!cfg || !bytes) return fail(MP_E_INVALID, "NULL argument");
  if (n_steps < 1) return fail(MP_E_INVALID, "n_steps must be >= 1");
  Geometry g;
  mp_status st = validate(prob, &g);
  if (st != MP_OK) return st;
  size_t po, ro;
  *bytes = align256(rve_bytes(layout(g, cfg->precision == MP_MIXED ? sizeof(float) : sizeof(double)),
                              n_steps, &po, &ro));
  return MP_OK;
}

mp_status mp_batch_create(const mp_batch_config* cfg, void* dev_workspace, size_t bytes,
                          void* hip_stream, mp_batch* out) {
  if (!cfg || !out) return fail(MP_E_INVALID, "NULL argument");
  if (cfg->precision != MP_FP64 && cfg->precision != MP_MIXED) return fail(MP_E_INVALID, "precision");
  if (cfg->n_shapes < 1 || cfg->n_shapes > kMaxClasses)
    return fail(MP_E_INVALID, "n_shapes must be 1.." + std::to_string(kMaxClasses));
  if (cfg->max_rves < 1 || cfg->max_rves > kMaxSlots)
    return fail(MP_E_INVALID, "max_rves must be 1.." + std::to_string(kMaxSlots));
  if (cfg->iters_per_launch < 1 || cfg->iters_per_launch > 64)
    return fail(MP_E_INVALID, "iters_per_launch must be 1..64");
  if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255))
    return fail(MP_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  for (int c = 0; c < cfg->n_shapes; ++c) {
    for (int i = 0; i < 3; ++i)
      if (!supported(cfg->shapes[c][i]))
        return fail(MP_E_INVALID, "unsupported shape class size " + std::to_string(cfg->shapes[c][i]));
    for (int d = 0; d < c; ++d)
      if (!std::memcmp(cfg->shapes[c], cfg->shapes[d], sizeof cfg->shapes[c]))
        return fail(MP_E_INVALID, "duplicate shape class");
  }
  const bool mixed = cfg->precision == MP_MIXED;
  const size_t rv_bytes = align256(size_t(kMaxSlots) * (mixed ? sizeof(Rve<float>) : sizeof(Rve<double>)));
  const size_t head = rv_bytes + align256(sizeof(Lists));
  if (bytes < head) return fail(MP_E_NOMEM, "workspace smaller than the batch's descriptors");

  mp_batch B = new mp_batch_s();
  B->cfg = *cfg;
  B->w = mixed ? sizeof(float) : sizeof(double);
  B->stream = reinterpret_cast<hipStream_t>(hip_stream);
  B->ws = static_cast<unsigned char*>(dev_workspace);
  B->bytes = bytes;
  B->arena.reset(bytes);
  size_t off;
  B->arena.alloc(head, &off);   // offset 0
  B->rv = B->ws + off;
  B->ls = reinterpret_cast<Lists*>(B->ws + off + rv_bytes);
  B->base_bytes = head;
  B->slot_id.assign(kMaxSlots, -1);
  B->next_id = 1;
  auto bail = [&](mp_status s) {
    if (B->ls_host) (void)hipHostFree(B->ls_host);
    if (B->ls_ahead) (void)hipHostFree(B->ls_ahead);
    for (hipEvent_t ev : B->drained)
      if (ev) (void)hipEventDestroy(ev);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
    return s;
  };
  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&B->ls_host), sizeof(Lists))) != hipSuccess ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&B->ls_ahead), offsetof(Lists, s))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&B->drained[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&B->drained[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking)) != hipSuccess ||
      (e = mixed ? BEng<float>::allow_all() : BEng<double>::allow_all()) != hipSuccess ||
      (e = hipMemsetAsync(B->ws, 0, head, B->stream)) != hipSuccess) {
    g_err = std::string("batch set-up: ") + hipGetErrorString(e);
    return bail(MP_E_DEVICE);
  }
  B->cls.resize(cfg->n_shapes);
  for (int c = 0; c < cfg->n_shapes; ++c) {
    ClassInfo& C = B->cls[c];
    for (int i = 0; i < 3; ++i) C.n[i] = cfg->shapes[c][i];
    C.g = grid_geometry(C.n[0], C.n[1], C.n[2]);
    mp_status st = mixed ? BEng<float>::setup_class(B, C) : BEng<double>::setup_class(B, C);
    if (st != MP_OK) return bail(st);
  }
  if ((e = hipStreamSynchronize(B->stream)) != hipSuccess) {
    g_err = std::string("batch set-up: ") + hipGetErrorString(e);
    return bail(MP_E_DEVICE);
  }
  *out = B;
  return MP_OK;
}

mp_status mp_batch_admit(mp_batch B, const mp_problem* prob, int32_t n_steps, const double* times,
                         const double* E, const double* Gam, int32_t* id) {
  if (!B || !id) return fail(MP_E_INVALID, "NULL argument");
  if (!prob || prob->precision != B->cfg.precision)
    return fail(MP_E_INVALID, "problem precision differs from the batch's");
  if (n_steps < 1 || !times || !E || !Gam) return fail(MP_E_INVALID, "bad load path");
  for (int s = 1; s <= n_steps; ++s)
    if (!(times[s] > times[s - 1])) return fail(MP_E_INVALID, "times must increase");
  for (int i = 0; i < 9 * n_steps; ++i)
    if (!std::isfinite(E[i]) || !std::isfinite(Gam[i])) return fail(MP_E_INVALID, "non-finite load");
  return B->w == sizeof(float) ? BEng<float>::admit(B, prob, n_steps, times, E, Gam, id)
                               : BEng<double>::admit(B, prob, n_steps, times, E, Gam, id);
}

mp_status mp_batch_run(mp_batch B, int32_t* n_active) {
  if (!B) return fail(MP_E_INVALID, "batch is NULL");
  mp_status st = capture(B);
  if (st != MP_OK) return st;
  HIP_TRY(hipGraphLaunch(B->exec, B->stream));
  HIP_TRY(hipMemcpyAsync(B->ls_host, B->ls, offsetof(Lists, s), hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->graph_launches += 1;
  if (n_active) *n_active = B->ls_host->active;
  return MP_OK;
}

// Graph launches until no RVE is unfinished.  After the first launch, the
// next launch is queued before the state after the previous one is read
// back, so the host's read-back and decision overlap the GPU's work instead
// of idling it between launches.  The launch queued after the last RVE
// finished runs on a finished batch: every work list is empty and the
// control leaves finished RVEs as they are, so it changes no result
// (*launches counts it).
mp_status mp_batch_drain(mp_batch B, int32_t max_launches, int32_t* launches) {
  if (!B) return fail(MP_E_INVALID, "batch is NULL");
  mp_status st = capture(B);
  if (st != MP_OK) return st;
  int32_t k = 0;
  Lists* const back[2] = {B->ls_host, B->ls_ahead};
  auto room = [&]() { return max_launches <= 0 || k < max_launches; };
  auto launch = [&](int b) -> mp_status {
    HIP_TRY(hipGraphLaunch(B->exec, B->stream));
    HIP_TRY(hipMemcpyAsync(back[b], B->ls, offsetof(Lists, s), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipEventRecord(B->drained[b], B->stream));
    B->graph_launches += 1;
    ++k;
    return MP_OK;
  };
  if (room()) {
    if ((st = launch(0)) != MP_OK) return st;
    HIP_TRY(hipEventSynchronize(B->drained[0]));
    if (back[0]->active > 0 && room()) {
      if ((st = launch(1)) != MP_OK) return st;
      for (int cur = 1;; cur ^= 1) {
        const bool ahead = room();
        if (ahead && (st = launch(cur ^ 1)) != MP_OK) return st;
        HIP_TRY(hipEventSynchronize(B->drained[cur]));
        if (back[cur]->active == 0 || !ahead) break;
      }
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
  }
  if (launches) *launches = k;
  return MP_OK;
}

mp_status mp_batch_query(mp_batch B, int32_t id, int32_t* state, int32_t* status, int32_t* steps_done,
                         int64_t* iters_total) {
  RveHost* H;
  mp_status st = find(B, id, &H);
  if (st != MP_OK) return st;
  int s, sc, c;
  long it;
  if ((st = query(B, *H, &s, &sc, &c, &it)) != MP_OK) return st;
  if (state) *state = s == RV_DONE ? MP_RVE_DONE : MP_RVE_RUNNING;
  if (status) *status = status_code(sc);
  if (steps_done) *steps_done = c;
  if (iters_total) *iters_total = it;
  return MP_OK;
}

mp_status mp_batch_response(mp_batch B, int32_t id, int32_t step, double out[48]) {
  RveHost* H;
  mp_status st = find(B, id, &H);
  if (st != MP_OK) return st;
  if (!out) return fail(MP_E_INVALID, "NULL argument");
  int s, sc, c;
  long it;
  if ((st = query(B, *H, &s, &sc, &c, &it)) != MP_OK) return st;
  if (step < 1 || step > c) return fail(MP_E_INVALID, "step not committed");
  double r[kRec];
  HIP_TRY(hipMemcpyAsync(r, B->ws + H->off + H->rec_off + size_t(step - 1) * kRec * sizeof(double),
                         sizeof r, hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (int j = 0; j < kNAvg; ++j) out[j] = r[j] / double(H->nvox);
  for (int j = kNAvg; j < kRec; ++j) out[j] = r[j];
  return MP_OK;
}

mp_status mp_batch_get_fields(mp_batch B, int32_t id, uint32_t mask, void* const* dst, int32_t dst_is_device) {
  RveHost* H;
  mp_status st = find(B, id, &H);
  if (st != MP_OK) return st;
  const unsigned char* b = B->ws + H->off;
  return copy_fields(b + H->L.E, b + H->L.out_tm, b + H->L.out_pq, H->nvox, B->w, mask, dst, dst_is_device,
                     B->stream);
}

mp_status mp_batch_set_fixed_iterations(mp_batch B, int32_t id, int32_t n_fixed) {
  RveHost* H;
  mp_status st = find(B, id, &H);
  if (st != MP_OK) return st;
  if (n_fixed < 0) return fail(MP_E_INVALID, "n_fixed < 0");
  // the descriptor's count (copied into the loop control at every step start)
  // and the running step's own
  const bool f32 = B->w == sizeof(float);
  const size_t base = size_t(H->slot) * (f32 ? sizeof(Rve<float>) : sizeof(Rve<double>));
  const size_t at_r = base + (f32 ? offsetof(Rve<float>, fixed) : offsetof(Rve<double>, fixed));
  const size_t at_c = base + (f32 ? offsetof(Rve<float>, ctl) : offsetof(Rve<double>, ctl)) +
                      offsetof(Ctl, fixed);
  unsigned char* d = static_cast<unsigned char*>(B->rv);
  HIP_TRY(hipMemcpyAsync(d + at_r, &n_fixed, sizeof n_fixed, hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipMemcpyAsync(d + at_c, &n_fixed, sizeof n_fixed, hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  return MP_OK;
}

mp_status mp_batch_release(mp_batch B, int32_t id) {
  RveHost* H;
  mp_status st = find(B, id, &H);
  if (st != MP_OK) return st;
  // empty the slot (a running RVE is cancelled) and drop it from the lists
  const int empty = RV_EMPTY;
  const size_t at = size_t(H->slot) * (B->w == sizeof(float) ? sizeof(Rve<float>) : sizeof(Rve<double>)) +
                    (B->w == sizeof(float) ? offsetof(Rve<float>, state) : offsetof(Rve<double>, state));
  HIP_TRY(hipMemcpyAsync(static_cast<unsigned char*>(B->rv) + at, &empty, sizeof empty,
                         hipMemcpyHostToDevice, B->stream));
  HIP_TRY(B->w == sizeof(float) ? BEng<float>::ctl(B, 0, B->stream) : BEng<double>::ctl(B, 0, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->arena.release(H->off, H->bytes);
  B->slot_id[H->slot] = -1;
  B->rves.erase(id);
  return MP_OK;
}

mp_status mp_batch_schedule(mp_batch B, int32_t cls, int32_t out[8], float ms[3]) {
  if (!B || !out) return fail(MP_E_INVALID, "NULL argument");
  if (cls < 0 || cls >= int(B->cls.size())) return fail(MP_E_INVALID, "class out of range");
  const ClassInfo& C = B->cls[cls];
  for (int p = 0; p < 3; ++p) {
    out[2 * p] = C.pass[p].tx;
    out[2 * p + 1] = C.pass[p].grid;
    if (ms) ms[p] = C.pass[p].ms;
  }
  out[6] = C.xgrid;
  out[7] = C.g.xblocks;
  return MP_OK;
}

mp_status mp_batch_stats(mp_batch B, int64_t* graph_launches, size_t* arena_used, int32_t* resident) {
  if (!B) return fail(MP_E_INVALID, "batch is NULL");
  if (graph_launches) *graph_launches = B->graph_launches;
  if (arena_used) *arena_used = B->arena.used();
  if (resident) *resident = int32_t(B->rves.size());
  return MP_OK;
}

void mp_batch_destroy(mp_batch B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->ls_host) (void)hipHostFree(B->ls_host);
  if (B->ls_ahead) (void)hipHostFree(B->ls_ahead);
  for (hipEvent_t ev : B->drained)
    if (ev) (void)hipEventDestroy(ev);
  delete B;
}

// ---------------------------------------------------------------------------
// serving loops
// ---------------------------------------------------------------------------
mp_status mp_serve_batched(mp_batch B, int32_t n, const mp_request* req, int32_t max_bypass,
                           double progress_s, double* t_admit, double* t_done, int32_t* status,
                           int64_t* iters) {
  if (!B || n < 0 || (n > 0 && (!req || !t_admit || !t_done || !status || !iters)))
    return fail(MP_E_INVALID, "bad argument");
  for (int i = 1; i < n; ++i)
    if (req[i].arrival < req[i - 1].arrival) return fail(MP_E_INVALID, "arrivals must be sorted");
  if (!B->rves.empty()) return fail(MP_E_STATE, "the batch must be empty");
  std::vector<int> queue;                 // arrived, not admitted, arrival order
  std::map<int32_t, int> running;         // RVE id -> request
  int next = 0, finished = 0, head_skips = 0;
  const double t0 = now_s();
  double last_note = t0;
  for (int i = 0; i < n; ++i) {
    t_admit[i] = t_done[i] = -1.0;
    status[i] = MP_OK;
    iters[i] = 0;
  }
  while (finished < n) {
    const double t = now_s() - t0;
    while (next < n && req[next].arrival <= t) queue.push_back(next++);
    if (progress_s > 0 && now_s() - last_note >= progress_s) {
      last_note = now_s();
      std::fprintf(stderr, "# serve t=%.1f s: %d done, %d running, %d queued, %d not arrived\n", t,
                   finished, int(running.size()), int(queue.size()), n - next);
      std::fflush(stderr);
    }
    // admission by footprint, arrival order; later requests may pass a head
    // that does not fit until the head has been passed max_bypass times
    for (size_t k = 0; k < queue.size();) {
      const int i = queue[k];
      mp_problem p = *req[i].prob;
      p.precision = B->cfg.precision;
      int32_t id;
      const mp_status st = mp_batch_admit(B, &p, req[i].n_steps, req[i].times, req[i].E, req[i].Gam, &id);
      if (st == MP_OK) {
        t_admit[i] = now_s() - t0;
        running[id] = i;
        queue.erase(queue.begin() + k);
        if (k == 0) head_skips = 0;
        else ++head_skips;
        continue;
      }
      if (st != MP_E_NOMEM) {   // invalid request: answered at once
        status[i] = st;
        t_admit[i] = t_done[i] = now_s() - t0;
        ++finished;
        queue.erase(queue.begin() + k);
        continue;
      }
      if (k == 0 && head_skips >= max_bypass) break;
      ++k;
    }
    if (running.empty()) {
      if (next < n) {
        double wait = req[next].arrival - (now_s() - t0);
        if (progress_s > 0) wait = std::min(wait, progress_s);
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      } else if (!queue.empty()) {
        return fail(MP_E_NOMEM, "a request does not fit in the empty arena");
      }
      continue;
    }
    int32_t active;
    mp_status st = mp_batch_run(B, &active);
    if (st != MP_OK) return st;
    // retire finished RVEs
    const Lists& ls = *B->ls_host;
    for (auto it = running.begin(); it != running.end();) {
      const RveHost& H = B->rves[it->first];
      if (ls.st[H.slot] != RV_DONE) {
        ++it;
        continue;
      }
      int s, sc, c;
      long itn;
      if ((st = query(B, H, &s, &sc, &c, &itn)) != MP_OK) return st;
      const int i = it->second;
      // the reply: the step records and the requested fields of the final
      // state, read back before the RVE's region is released
      if (req[i].records && (st = read_records(B, H, c, req[i].records)) != MP_OK) return st;
      if (req[i].field_mask &&
          (st = mp_batch_get_fields(B, it->first, req[i].field_mask, req[i].fields, req[i].fields_on_device)) !=
              MP_OK)
        return st;
      if (req[i].field_mask && req[i].fields_on_device) HIP_TRY(hipStreamSynchronize(B->stream));
      t_done[i] = now_s() - t0;
      status[i] = status_code(sc);
      iters[i] = itn;
      if ((st = mp_batch_release(B, it->first)) != MP_OK) return st;
      it = running.erase(it);
      ++finished;
    }
  }
  return MP_OK;
}

mp_status mp_serve_sequential(int32_t n, const mp_request* req, void* dev_workspace, size_t bytes,
                              void* hip_stream, double progress_s, double* t_start, double* t_done,
                              int32_t* status, int64_t* iters) {
  if (n < 0 || (n > 0 && (!req || !t_start || !t_done || !status || !iters)))
    return fail(MP_E_INVALID, "bad argument");
  for (int i = 1; i < n; ++i)
    if (req[i].arrival < req[i - 1].arrival) return fail(MP_E_INVALID, "arrivals must be sorted");
  const double t0 = now_s();
  double last_note = t0;
  for (int i = 0; i < n; ++i) {
    for (;;) {   // wait for the arrival (in slices when reporting progress)
      double wait = req[i].arrival - (now_s() - t0);
      if (wait <= 0) break;
      if (progress_s > 0) wait = std::min(wait, progress_s);
      std::this_thread::sleep_for(std::chrono::duration<double>(wait));
    }
    t_start[i] = now_s() - t0;
    mp_problem p = *req[i].prob;
    p.precision = MP_FP64;
    size_t need;
    mp_status st = mp_plan_workspace_size(&p, &need);
    if (st == MP_OK && need > bytes) st = fail(MP_E_NOMEM, "request larger than the workspace");
    mp_plan P = nullptr;
    if (st == MP_OK) st = mp_plan_create(&p, dev_workspace, bytes, hip_stream, &P);
    std::vector<int32_t> it(std::max(1, req[i].n_steps), 0);
    // one step per call (the plan continues from its committed state), so
    // progress can be reported between steps
    for (int k = 0; st == MP_OK && k < req[i].n_steps; ++k) {
      st = mp_solve_load_path(P, 1, req[i].times + k, req[i].E + 9 * k, req[i].Gam + 9 * k, &it[k]);
      if (progress_s > 0 && now_s() - last_note >= progress_s) {
        last_note = now_s();
        std::fprintf(stderr, "# sequential t=%.1f s: request %d of %d, step %d of %d\n", last_note - t0,
                     i + 1, n, k + 1, req[i].n_steps);
        std::fflush(stderr);
      }
    }
    // the reply: step records and requested fields, before the plan goes
    if (P && st != MP_E_DEVICE) {
      int32_t done_steps = 0;
      mp_plan_steps(P, &done_steps);
      if (req[i].records) {
        for (int k = 0; k < req[i].n_steps; ++k) {
          double* r = req[i].records + size_t(k) * kRec;
          if (k >= done_steps) {
            for (int j = 0; j < kRec; ++j) r[j] = std::nan("");
            continue;
          }
          mp_homogenized_response(P, k + 1, r);
          mp_step_error_parts(P, k + 1, r + 42);
          r[47] = 0.0;
        }
      }
      if (req[i].field_mask) {
        const mp_status fs = mp_get_fields(P, req[i].field_mask, req[i].fields, req[i].fields_on_device);
        if (fs == MP_OK && req[i].fields_on_device) (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream));
        if (fs != MP_OK && st == MP_OK) st = fs;
      }
    }
    if (P) mp_plan_destroy(P);
    long tot = 0;
    for (int32_t v : it) tot += v;
    iters[i] = tot;
    status[i] = st;
    t_done[i] = now_s() - t0;
    if (progress_s > 0) {
      std::fprintf(stderr, "# sequential t=%.1f s: request %d of %d done (%ld iterations)\n",
                   t_done[i], i + 1, n, tot);
      std::fflush(stderr);
    }
    if (st == MP_E_DEVICE) return st;
  }
  return MP_OK;
}

}  // extern "C"
