// Host side of the micropolar FFT solver: plan, workspace layout, Alg. 2
// step loop and the C ABI declared in include/mp.h.
#include "../../include/mp.h"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace mp;

namespace {

thread_local std::string g_err;

mp_status fail(mp_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(MP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

// ---------------------------------------------------------------------------
// compile-time sizes: every axis length must be one of these
// ---------------------------------------------------------------------------
#define MP_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

bool supported(int n) {
  switch (n) {
#define MP_CASE(N) case N:
    MP_SIZES(MP_CASE)
#undef MP_CASE
    return true;
    default: return false;
  }
}

// widest y / z tile: TX * L <= 256 frequencies (a power of two)
constexpr int tx_wide(int L) {
  int t = 1;
  while (2 * t * L <= 256) t *= 2;
  return t;
}

int x_rows(int n0) { return n0 >= 128 ? 1 : 128 / n0; }

template <class T, int MODE>
void launch_x(int n0, int blocks, hipStream_t s, const XArgs<T>& a) {
  switch (n0) {
#define MP_CASE(N)                                                                           \
  case N:                                                                                    \
    hipLaunchKernelGGL((k_xpass<T, MODE, N>), dim3(blocks), dim3(XShape<N>::NTHR), 0, s, a); \
    break;
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
}

template <class T, int MODE, int L, int TX>
void launch_axis_tx(dim3 grid, hipStream_t s, const AxisArgs<T>& a) {
  const size_t shm = size_t(AShape<L, TX>::PTS) * sizeof(cx<T>);
  hipLaunchKernelGGL((k_axis<T, MODE, L, TX>), grid, dim3(AShape<L, TX>::NTHR), shm, s, a);
}

template <class T, int MODE>
void launch_axis(int L, int tx, dim3 grid, hipStream_t s, const AxisArgs<T>& a) {
  switch (L) {
#define MP_CASE(N)                                        \
  case N:                                                 \
    if (tx == 1)                                          \
      launch_axis_tx<T, MODE, N, 1>(grid, s, a);          \
    else                                                  \
      launch_axis_tx<T, MODE, N, tx_wide(N)>(grid, s, a); \
    break;
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
}

// let every axis kernel use more than 64 KB of LDS (up to 160 KB on gfx950)
template <class T, int MODE, int L, int TX>
hipError_t allow_lds_tx() {
  const size_t shm = size_t(AShape<L, TX>::PTS) * sizeof(cx<T>);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_axis<T, MODE, L, TX>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
}

template <class T, int MODE>
hipError_t allow_lds(int L) {
  hipError_t e = hipSuccess;
  switch (L) {
#define MP_CASE(N)                                                   \
  case N:                                                            \
    if ((e = allow_lds_tx<T, MODE, N, 1>()) != hipSuccess) return e; \
    e = allow_lds_tx<T, MODE, N, tx_wide(N)>();                      \
    break;
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
  return e;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t S, E, Eprev, base, pq, out_tm, out_pq, phase, params, tw, partials, ctl, tot, resp, total;
};

struct Geometry {
  int n0, n1, n2, nh;
  long nvox, nspec, nrows;
  int xblocks, txy, txz;
  int commit_blocks;
};

constexpr int kProfEv = 6;     // boundaries around the 5 loop kernels of one iteration
constexpr int kFloorWindow = 100;

}  // namespace

struct mp_plan_s {
  Geometry g;
  Layout L;
  int precision;
  double h;
  hipStream_t stream;
  unsigned char* ws;
  void* S;        // cx<T>
  void* E;        // T
  void* Eprev;    // T
  void* base;     // T
  void* out_tm;   // T
  double *pq, *out_pq, *partials, *tot, *resp;
  uint8_t* phase;
  PhaseC* params;
  void* tw0;      // cx<T>, n0 + n1 + n2 entries
  Ctl* ctl;
  Ctl* ctl_host;
  RefC ref;
  double tol;
  int max_iter, norm, fixed;
  int n_phases;
  int steps;
  double t_prev, t_cur;   // times of the last two committed states
  std::vector<std::vector<double>> resp_hist;
  // optional per-kernel timing of loop iterations (hipEvents on the plan's stream)
  bool prof;
  std::vector<hipEvent_t> ev;
  double prof_ms[8];
  long prof_n[8];
};

namespace {

mp_status validate(const mp_problem* p, Geometry* g) {
  if (!p) return fail(MP_E_INVALID, "problem is NULL");
  for (int i = 0; i < 3; ++i)
    if (!supported(p->n[i]))
      return fail(MP_E_INVALID, "grid size n[" + std::to_string(i) + "] = " + std::to_string(p->n[i]) +
                                    " unsupported (4 6 8 12 16 24 32 48 64 96 128 192 256)");
  if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(MP_E_INVALID, "h must be > 0");
  if (p->n_phases < 1 || p->n_phases > 256) return fail(MP_E_INVALID, "n_phases out of 1..256");
  if (!p->phase || !p->phases) return fail(MP_E_INVALID, "phase map / table is NULL");
  if (!(p->tol > 0.0)) return fail(MP_E_INVALID, "tol must be > 0");
  if (p->max_iter < 1) return fail(MP_E_INVALID, "max_iter must be >= 1");
  if (p->err_norm != MP_ERR_LOCAL && p->err_norm != MP_ERR_AVERAGE)
    return fail(MP_E_INVALID, "err_norm");
  if (p->precision != MP_FP64 && p->precision != MP_MIXED) return fail(MP_E_INVALID, "precision");
  if (p->ref_mode < 0 || p->ref_mode > 2) return fail(MP_E_INVALID, "ref_mode");
  for (int i = 0; i < p->n_phases; ++i) {
    const mp_phase& c = p->phases[i];
    const std::string tag = "phase " + std::to_string(i) + ": ";
    const double v[12] = {c.lambda, c.mu, c.kappa, c.alpha, c.beta, c.gamma,
                          c.tY, c.tH, c.mY, c.mH, c.a1, c.b1};
    for (int k = 0; k < 12; ++k)
      if (std::isnan(v[k])) return fail(MP_E_INVALID, tag + "NaN constant");
    // Eq. 7 energetic bounds (gamma - beta = 0 accepted)
    if (!(3 * c.lambda + 2 * c.mu > 0) || !(c.mu > 0) || !(c.kappa > 0) ||
        !(3 * c.alpha + c.beta + c.gamma > 0) || !(c.gamma + c.beta > 0) || !(c.gamma - c.beta >= 0))
      return fail(MP_E_INVALID, tag + "energetic bounds violated");
    if (!(c.tY > 0) || !(c.mY > 0)) return fail(MP_E_INVALID, tag + "yield stresses must be > 0");
    if (!(c.tH >= 0) || !(c.mH >= 0) || !std::isfinite(c.tH) || !std::isfinite(c.mH))
      return fail(MP_E_INVALID, tag + "hardening moduli must be finite and >= 0");
    if (!(c.a1 > 0) || !(c.b1 > 0) || !std::isfinite(c.a1) || !std::isfinite(c.b1))
      return fail(MP_E_INVALID, tag + "a1, b1 must be finite and > 0");
    if (std::isfinite(c.mY) && c.alpha != 0.0)
      return fail(MP_E_INVALID, tag + "micro-plastic phases need alpha = 0");
    for (int k = 0; k < 6; ++k)
      if (!std::isfinite(v[k])) return fail(MP_E_INVALID, tag + "moduli must be finite");
  }
  const long nvox = long(p->n[0]) * p->n[1] * p->n[2];
  for (long i = 0; i < nvox; ++i)
    if (p->phase[i] >= p->n_phases) return fail(MP_E_INVALID, "phase id out of range");

  Geometry G{};
  G.n0 = p->n[0]; G.n1 = p->n[1]; G.n2 = p->n[2]; G.nh = G.n0 / 2;
  G.nvox = nvox;
  G.nspec = long(G.n2) * G.n1 * G.nh;
  G.nrows = long(G.n1) * G.n2;
  const int rows = x_rows(G.n0);
  G.xblocks = int((G.nrows + rows - 1) / rows);
  G.txy = (G.nh % tx_wide(G.n1) == 0) ? tx_wide(G.n1) : 1;
  G.txz = (G.nh % tx_wide(G.n2) == 0) ? tx_wide(G.n2) : 1;
  G.commit_blocks = int((nvox + 255) / 256);
  *g = G;
  return MP_OK;
}

Layout layout(const Geometry& g, size_t w /* bytes per bulk word */) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.S = take(18 * g.nspec * 2 * w);
  L.E = take(18 * g.nvox * w);
  L.Eprev = take(18 * g.nvox * w);
  L.base = take(18 * g.nvox * w);
  L.pq = take(2 * g.nvox * sizeof(double));
  L.out_tm = take(18 * g.nvox * w);
  L.out_pq = take(2 * g.nvox * sizeof(double));
  L.phase = take(g.nvox);
  L.params = take(256 * sizeof(PhaseC));
  L.tw = take(size_t(g.n0 + g.n1 + g.n2) * 2 * w);
  L.partials = take(size_t(std::max(g.xblocks * kNPart, g.commit_blocks * kNAvg)) * sizeof(double));
  L.ctl = take(sizeof(Ctl));
  L.tot = take(32 * sizeof(double));
  L.resp = take(64 * sizeof(double));
  L.total = o;
  return L;
}

PhaseC derive(const mp_phase& c) {
  PhaseC d{};
  d.t.lam = c.lambda; d.t.mu = c.mu; d.t.kap = c.kappa;
  d.t.tY = c.tY; d.t.tH = c.tH; d.t.a1 = c.a1;
  d.t.a2 = c.a1 * c.mu / c.kappa;
  d.m.alp = c.alpha; d.m.bet = c.beta; d.m.gam = c.gamma;
  d.m.mY = c.mY; d.m.mH = c.mH; d.m.b1 = c.b1;
  if (c.gamma != c.beta) {
    d.m.b2 = c.b1 * (c.gamma + c.beta) / (c.gamma - c.beta);
    d.m.b2gmb = d.m.b2 * (c.gamma - c.beta);
  } else {
    d.m.b2 = 0.0;
    d.m.b2gmb = c.b1 * (c.gamma + c.beta);
  }
  return d;
}

template <class T>
void twiddles(int n, std::vector<cx<T>>* out) {
  for (int m = 0; m < n; ++m) {
    // exp(-2 pi i m / n), evaluated in long double
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * m / n;
    out->push_back(cx<T>{T(cosl(a)), T(sinl(a))});
  }
}

// ---------------------------------------------------------------------------
// typed launch helpers
// ---------------------------------------------------------------------------
template <class T>
struct Eng {
  static cx<T>* S(mp_plan P) { return static_cast<cx<T>*>(P->S); }
  static const cx<T>* tw(mp_plan P, int axis) {
    const cx<T>* t = static_cast<const cx<T>*>(P->tw0);
    return axis == 0 ? t : axis == 1 ? t + P->g.n0 : t + P->g.n0 + P->g.n1;
  }

  static AxisArgs<T> yargs(mp_plan P, cx<T>* S, const Ctl* ctl) {
    const Geometry& g = P->g;
    AxisArgs<T> a{};
    a.S = S;
    a.ostride = long(g.n1) * g.nh * 18;   // one kz plane
    a.pstride = long(g.nh) * 18;          // next ky
    a.tw = tw(P, 1);
    a.ctl = ctl;
    return a;
  }
  static AxisArgs<T> zargs(mp_plan P, cx<T>* S, const Ctl* ctl) {
    const Geometry& g = P->g;
    AxisArgs<T> a{};
    a.S = S;
    a.ostride = long(g.nh) * 18;          // next ky
    a.pstride = long(g.n1) * g.nh * 18;   // next kz
    a.tw = tw(P, 2);
    a.ctl = ctl;
    a.n0 = g.n0; a.n1 = g.n1; a.n2 = g.n2;
    a.h = P->h;
    a.scale = 1.0 / double(g.nvox);
    a.ref = P->ref;
    return a;
  }
  static dim3 ygrid(const Geometry& g) { return dim3(g.nh / g.txy, g.n2); }
  static dim3 zgrid(const Geometry& g) { return dim3(g.nh / g.txz, g.n1); }

  // y fwd, z fwd + Green + z inv, y inv (ev: optional events before each
  // kernel and after the last)
  static void spectral(mp_plan P, cx<T>* S, const Ctl* ctl, hipEvent_t* ev) {
    const Geometry& g = P->g;
    auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], P->stream); };
    const AxisArgs<T> ay = yargs(P, S, ctl), az = zargs(P, S, ctl);
    mark(0);
    launch_axis<T, Y_FWD>(g.n1, g.txy, ygrid(g), P->stream, ay);
    mark(1);
    launch_axis<T, Z_GREEN>(g.n2, g.txz, zgrid(g), P->stream, az);
    mark(2);
    launch_axis<T, Y_INV>(g.n1, g.txy, ygrid(g), P->stream, ay);
    mark(3);
  }

  static XArgs<T> xargs(mp_plan P) {
    const Geometry& g = P->g;
    XArgs<T> a{};
    a.nrows = g.nrows;
    a.tw = tw(P, 0);
    a.S = S(P);
    a.nvox = g.nvox;
    a.E = static_cast<T*>(P->E);
    a.Eprev = static_cast<T*>(P->Eprev);
    a.base = static_cast<const T*>(P->base);
    a.pq = P->pq;
    a.phase = P->phase;
    a.params = P->params;
    a.partials = P->partials;
    a.ctl = P->ctl;
    a.ref = P->ref;
    return a;
  }

  static hipError_t prepare() {
    hipError_t e;
    const int sizes[] = {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    for (int L : sizes) {
      if ((e = allow_lds<T, Y_FWD>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Y_INV>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_GREEN>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_FWD>(L)) != hipSuccess) return e;
    }
    return hipSuccess;
  }

  static mp_status solve(mp_plan P, int32_t n_steps, const double* times, const double* E,
                         const double* Gam, int32_t* iters);
};

template <class T>
mp_status Eng<T>::solve(mp_plan P, int32_t n_steps, const double* times, const double* E,
                        const double* Gam, int32_t* iters) {
  const Geometry& g = P->g;
  if (P->steps == 0) P->t_prev = P->t_cur = times[0];
  for (int s = 1; s <= n_steps; ++s) {
    XArgs<T> xa = xargs(P);
    for (int c = 0; c < 9; ++c) {
      xa.mac[c] = E[(s - 1) * 9 + c];
      xa.mac[9 + c] = Gam[(s - 1) * 9 + c];
    }
    xa.first = P->steps == 0;
    // Alg. 2 linear extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
    xa.r = P->steps == 0 ? 0.0 : (times[s] - P->t_cur) / (P->t_cur - P->t_prev);
    // the low-precision form may stop at its rounding floor: no new best
    // error for kFloorWindow iterations (flagged in the step record)
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, P->stream, P->ctl, P->fixed, P->max_iter,
                       P->tol, P->norm, sizeof(T) < sizeof(double) ? kFloorWindow : 0);
    P->ctl_host->iters = 0;
    P->ctl_host->done = 0;
    // first iterate (extrapolated or uniform), its return map and polarization
    xa.ctl = nullptr;
    launch_x<T, X_INIT>(g.n0, g.xblocks, P->stream, xa);
    xa.ctl = P->ctl;
    ErrMacro em;
    for (int c = 0; c < 18; ++c) em.v[c] = xa.mac[c];
    int batch = 2;
    long queued = 0;
    for (;;) {
      // the control block ends every step within max_iter (or the fixed count)
      // iterations; a loop that runs far past that means a broken device state
      if (queued > long(std::max(P->max_iter, P->fixed)) + 256)
        return fail(MP_E_DEVICE, "iteration control did not finish the step");
      queued += batch;
      const int it0 = P->ctl_host->iters;
      if (P->prof && P->ev.size() < size_t(batch) * kProfEv) {
        const size_t old = P->ev.size();
        P->ev.resize(size_t(batch) * kProfEv);
        for (size_t i = old; i < P->ev.size(); ++i) HIP_TRY(hipEventCreate(&P->ev[i]));
      }
      for (int k = 0; k < batch; ++k) {
        hipEvent_t* ev = P->prof ? &P->ev[size_t(k) * kProfEv] : nullptr;
        spectral(P, S(P), P->ctl, ev);
        launch_x<T, X_ITER>(g.n0, g.xblocks, P->stream, xa);
        if (ev) HIP_TRY(hipEventRecord(ev[4], P->stream));
        hipLaunchKernelGGL(k_err_rows, dim3(kNPart), dim3(256), 0, P->stream, P->partials, g.xblocks,
                           P->tot, P->ctl);
        hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, P->stream, P->tot, g.nvox, P->ctl, em);
        if (ev) HIP_TRY(hipEventRecord(ev[5], P->stream));
      }
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(P->ctl_host, P->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
      HIP_TRY(hipStreamSynchronize(P->stream));
      if (P->prof) {
        // only iterations that really ran (later ones returned at once)
        const int ran = std::min(batch, P->ctl_host->iters - it0);
        for (int k = 0; k < ran; ++k)
          for (int j = 0; j < kProfEv - 1; ++j) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, P->ev[size_t(k) * kProfEv + j],
                                        P->ev[size_t(k) * kProfEv + j + 1]));
            P->prof_ms[j] += ms;
            P->prof_n[j] += 1;
          }
      }
      if (P->ctl_host->done) break;
      batch = std::min(batch * 2, 64);
    }
    const Ctl c = *P->ctl_host;
    // commit
    CommitArgs<T> ca{g.nvox, static_cast<const T*>(P->E), static_cast<T*>(P->base), P->pq,
                     static_cast<T*>(P->out_tm), P->out_pq, P->phase, P->params, P->partials};
    hipLaunchKernelGGL((k_commit<T>), dim3(g.commit_blocks), dim3(256), 0, P->stream, ca);
    hipLaunchKernelGGL(k_avg_reduce, dim3(1), dim3(256), 0, P->stream, P->partials, g.commit_blocks,
                       g.nvox, P->resp);
    std::vector<double> r(47, 0.0);
    HIP_TRY(hipMemcpyAsync(r.data(), P->resp, kNAvg * sizeof(double), hipMemcpyDeviceToHost,
                           P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    r[40] = c.err;
    r[41] = c.iters;
    for (int f = 0; f < 4; ++f) r[42 + f] = c.err_parts[f];
    r[46] = c.done == 4 ? 1.0 : 0.0;
    P->resp_hist.push_back(r);
    P->steps += 1;
    P->t_prev = P->t_cur;
    P->t_cur = times[s];
    if (iters) iters[s - 1] = c.iters;
    if (c.done == 2)
      return fail(MP_E_NOT_CONVERGED, "step " + std::to_string(P->steps) + " hit max_iter");
    if (c.done == 3)
      return fail(MP_E_DIVERGED, "step " + std::to_string(P->steps) + " diverged");
  }
  return MP_OK;
}

}  // namespace

extern "C" {

const char* mp_last_error(void) { return g_err.c_str(); }
const char* mp_version(void) { return "mp 0.2 gfx950"; }

mp_status mp_plan_workspace_size(const mp_problem* prob, size_t* bytes) {
  Geometry g;
  mp_status s = validate(prob, &g);
  if (s != MP_OK) return s;
  if (!bytes) return fail(MP_E_INVALID, "bytes is NULL");
  *bytes = layout(g, prob->precision == MP_MIXED ? sizeof(float) : sizeof(double)).total;
  return MP_OK;
}

mp_status mp_plan_create(const mp_problem* prob, void* dev_workspace, size_t bytes, void* hip_stream,
                         mp_plan* out) {
  Geometry g;
  mp_status s = validate(prob, &g);
  if (s != MP_OK) return s;
  if (!out) return fail(MP_E_INVALID, "out is NULL");
  const bool mixed = prob->precision == MP_MIXED;
  const size_t w = mixed ? sizeof(float) : sizeof(double);
  Layout L = layout(g, w);
  if (!dev_workspace || bytes < L.total)
    return fail(MP_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255)
    return fail(MP_E_INVALID, "workspace must be 256-byte aligned");

  mp_plan P = new mp_plan_s();
  P->g = g;
  P->L = L;
  P->precision = prob->precision;
  P->h = prob->h;
  P->stream = reinterpret_cast<hipStream_t>(hip_stream);
  unsigned char* wsp = static_cast<unsigned char*>(dev_workspace);
  P->ws = wsp;
  P->S = wsp + L.S;
  P->E = wsp + L.E;
  P->Eprev = wsp + L.Eprev;
  P->base = wsp + L.base;
  P->pq = reinterpret_cast<double*>(wsp + L.pq);
  P->out_tm = wsp + L.out_tm;
  P->out_pq = reinterpret_cast<double*>(wsp + L.out_pq);
  P->phase = wsp + L.phase;
  P->params = reinterpret_cast<PhaseC*>(wsp + L.params);
  P->tw0 = wsp + L.tw;
  P->partials = reinterpret_cast<double*>(wsp + L.partials);
  P->ctl = reinterpret_cast<Ctl*>(wsp + L.ctl);
  P->tot = reinterpret_cast<double*>(wsp + L.tot);
  P->resp = reinterpret_cast<double*>(wsp + L.resp);
  P->tol = prob->tol;
  P->max_iter = prob->max_iter;
  P->norm = prob->err_norm;
  P->fixed = 0;
  P->prof = false;
  for (int j = 0; j < 8; ++j) { P->prof_ms[j] = 0.0; P->prof_n[j] = 0; }
  P->n_phases = prob->n_phases;
  P->steps = 0;
  P->t_prev = P->t_cur = 0.0;

  // reference medium (Alg. 2: A0 = <A>, B0 = <B>); phase mean by default
  double refv[6] = {0, 0, 0, 0, 0, 0};
  if (prob->ref_mode == MP_REF_EXPLICIT) {
    const mp_phase& r = prob->ref;
    const double v[6] = {r.lambda, r.mu, r.kappa, r.alpha, r.beta, r.gamma};
    std::memcpy(refv, v, sizeof v);
  } else {
    std::vector<long> count(prob->n_phases, 0);
    for (long i = 0; i < g.nvox; ++i) count[prob->phase[i]]++;
    double wsum = 0;
    for (int i = 0; i < prob->n_phases; ++i) {
      if (!count[i]) continue;
      const double wgt = prob->ref_mode == MP_REF_VOLUME_MEAN ? double(count[i]) : 1.0;
      const mp_phase& c = prob->phases[i];
      const double v[6] = {c.lambda, c.mu, c.kappa, c.alpha, c.beta, c.gamma};
      for (int k = 0; k < 6; ++k) refv[k] += wgt * v[k];
      wsum += wgt;
    }
    for (int k = 0; k < 6; ++k) refv[k] /= wsum;
  }
  P->ref = RefC{refv[0], refv[1], refv[2], refv[3], refv[4], refv[5]};
  if (!(P->ref.lam + 2 * P->ref.mu > 0) || !(P->ref.mu > 0) || !(P->ref.kap > 0) ||
      !(P->ref.gam > 0) || !(P->ref.alp + P->ref.bet + P->ref.gam > 0)) {
    delete P;
    return fail(MP_E_INVALID, "reference medium is not positive definite");
  }

  std::vector<PhaseC> pc(256);
  for (int i = 0; i < prob->n_phases; ++i) pc[i] = derive(prob->phases[i]);
  std::vector<cx<double>> tw;
  std::vector<cx<float>> twf;
  if (mixed) {
    twiddles(g.n0, &twf);
    twiddles(g.n1, &twf);
    twiddles(g.n2, &twf);
  } else {
    twiddles(g.n0, &tw);
    twiddles(g.n1, &tw);
    twiddles(g.n2, &tw);
  }

  auto cleanup = [&](mp_status st) { delete P; return st; };
  hipError_t e;
#define CREATE_TRY(call)                                                                 \
  do {                                                                                   \
    if ((e = (call)) != hipSuccess) {                                                    \
      g_err = std::string(#call) + ": " + hipGetErrorString(e);                          \
      return cleanup(MP_E_DEVICE);                                                       \
    }                                                                                    \
  } while (0)
  CREATE_TRY(mixed ? Eng<float>::prepare() : Eng<double>::prepare());
  CREATE_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->ctl_host), sizeof(Ctl)));
  CREATE_TRY(hipMemsetAsync(wsp, 0, L.total, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->phase, prob->phase, g.nvox, hipMemcpyHostToDevice, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->params, pc.data(), pc.size() * sizeof(PhaseC), hipMemcpyHostToDevice,
                            P->stream));
  if (mixed) {
    CREATE_TRY(hipMemcpyAsync(P->tw0, twf.data(), twf.size() * sizeof(cx<float>),
                              hipMemcpyHostToDevice, P->stream));
  } else {
    CREATE_TRY(hipMemcpyAsync(P->tw0, tw.data(), tw.size() * sizeof(cx<double>),
                              hipMemcpyHostToDevice, P->stream));
  }
  CREATE_TRY(hipStreamSynchronize(P->stream));
#undef CREATE_TRY
  *out = P;
  return MP_OK;
}

void mp_plan_destroy(mp_plan P) {
  if (!P) return;
  if (P->ctl_host) (void)hipHostFree(P->ctl_host);
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  delete P;
}

mp_status mp_profile(mp_plan P, int32_t enable) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  P->prof = enable != 0;
  for (int j = 0; j < 8; ++j) {
    P->prof_ms[j] = 0.0;
    P->prof_n[j] = 0;
  }
  return MP_OK;
}

mp_status mp_profile_read(mp_plan P, int32_t n, double* ms_total, int64_t* launches) {
  if (!P || !ms_total || !launches || n < 0) return fail(MP_E_INVALID, "bad argument");
  for (int j = 0; j < n && j < kProfEv - 1; ++j) {
    ms_total[j] = P->prof_ms[j];
    launches[j] = P->prof_n[j];
  }
  return MP_OK;
}

mp_status mp_set_fixed_iterations(mp_plan P, int32_t n_fixed) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  if (n_fixed < 0) return fail(MP_E_INVALID, "n_fixed < 0");
  P->fixed = n_fixed;
  return MP_OK;
}

mp_status mp_plan_steps(mp_plan P, int32_t* steps) {
  if (!P || !steps) return fail(MP_E_INVALID, "NULL argument");
  *steps = P->steps;
  return MP_OK;
}

mp_status mp_solve_load_path(mp_plan P, int32_t n_steps, const double* times, const double* E,
                             const double* Gam, int32_t* iters) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  if (n_steps < 0 || (n_steps > 0 && (!times || !E || !Gam)))
    return fail(MP_E_INVALID, "bad load path");
  if (n_steps == 0) return MP_OK;
  if (P->steps > 0 && times[0] != P->t_cur)
    return fail(MP_E_STATE, "times[0] must equal the time of the last committed step");
  for (int s = 1; s <= n_steps; ++s)
    if (!(times[s] > times[s - 1])) return fail(MP_E_INVALID, "times must increase");
  for (int i = 0; i < 9 * n_steps; ++i)
    if (!std::isfinite(E[i]) || !std::isfinite(Gam[i])) return fail(MP_E_INVALID, "non-finite load");
  if (P->precision == MP_MIXED) return Eng<float>::solve(P, n_steps, times, E, Gam, iters);
  return Eng<double>::solve(P, n_steps, times, E, Gam, iters);
}

mp_status mp_homogenized_response(mp_plan P, int32_t step, double out[42]) {
  if (!P || !out) return fail(MP_E_INVALID, "NULL argument");
  if (step < 1 || step > P->steps) return fail(MP_E_INVALID, "step out of range");
  std::memcpy(out, P->resp_hist[step - 1].data(), 42 * sizeof(double));
  return MP_OK;
}

mp_status mp_step_error_parts(mp_plan P, int32_t step, double out[5]) {
  if (!P || !out) return fail(MP_E_INVALID, "NULL argument");
  if (step < 1 || step > P->steps) return fail(MP_E_INVALID, "step out of range");
  std::memcpy(out, P->resp_hist[step - 1].data() + 42, 5 * sizeof(double));
  return MP_OK;
}

mp_status mp_get_fields(mp_plan P, int32_t field, double* dst) {
  if (!P || !dst) return fail(MP_E_INVALID, "NULL argument");
  const long n = P->g.nvox;
  const size_t w = P->precision == MP_MIXED ? sizeof(float) : sizeof(double);
  const unsigned char* src = nullptr;
  long count = 9 * n;
  bool bulk = true;   // stored in the bulk type (else FP64)
  switch (field) {
    case MP_FIELD_E: src = static_cast<const unsigned char*>(P->E); break;
    case MP_FIELD_GAMMA: src = static_cast<const unsigned char*>(P->E) + 9 * n * w; break;
    case MP_FIELD_T: src = static_cast<const unsigned char*>(P->out_tm); break;
    case MP_FIELD_M: src = static_cast<const unsigned char*>(P->out_tm) + 9 * n * w; break;
    case MP_FIELD_P: src = reinterpret_cast<const unsigned char*>(P->out_pq); count = n; bulk = false; break;
    case MP_FIELD_Q: src = reinterpret_cast<const unsigned char*>(P->out_pq + n); count = n; bulk = false; break;
    default: return fail(MP_E_INVALID, "unknown field");
  }
  if (bulk && w == sizeof(float)) {
    std::vector<float> tmp(count);
    HIP_TRY(hipMemcpyAsync(tmp.data(), src, count * sizeof(float), hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    for (long i = 0; i < count; ++i) dst[i] = double(tmp[i]);
    return MP_OK;
  }
  HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

mp_status mp_spectrum_forward(mp_plan P, const void* dev_in, void* dev_out) {
  if (!P || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  if (P->precision != MP_FP64) return fail(MP_E_INVALID, "FP64 plans only");
  using E8 = Eng<double>;
  const Geometry& g = P->g;
  XArgs<double> xa = E8::xargs(P);
  xa.ctl = nullptr;
  xa.fin = static_cast<const double*>(dev_in);
  cx<double>* S = static_cast<cx<double>*>(dev_out);
  xa.S = S;
  launch_x<double, X_FWD_ONLY>(g.n0, g.xblocks, P->stream, xa);
  launch_axis<double, Y_FWD>(g.n1, g.txy, E8::ygrid(g), P->stream, E8::yargs(P, S, nullptr));
  launch_axis<double, Z_FWD>(g.n2, g.txz, E8::zgrid(g), P->stream, E8::zargs(P, S, nullptr));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

mp_status mp_green_apply(mp_plan P, const void* dev_in, void* dev_out) {
  if (!P || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  if (P->precision != MP_FP64) return fail(MP_E_INVALID, "FP64 plans only");
  using E8 = Eng<double>;
  const Geometry& g = P->g;
  XArgs<double> xa = E8::xargs(P);
  xa.ctl = nullptr;
  xa.fin = static_cast<const double*>(dev_in);
  launch_x<double, X_FWD_ONLY>(g.n0, g.xblocks, P->stream, xa);
  E8::spectral(P, E8::S(P), nullptr, nullptr);
  xa.fout = static_cast<double*>(dev_out);
  launch_x<double, X_INV_ONLY>(g.n0, g.xblocks, P->stream, xa);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

mp_status mp_radial_return(mp_plan P, int64_t n, const void* phase, const void* e, const void* g,
                           const void* e_n, const void* g_n, const void* t_n, const void* m_n,
                           const void* p_n, const void* q_n, void* t, void* m, void* p, void* q) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  if (n < 0) return fail(MP_E_INVALID, "n < 0");
  if (n == 0) return MP_OK;
  if (!phase || !e || !g || !e_n || !g_n || !t_n || !m_n || !p_n || !q_n || !t || !m || !p || !q)
    return fail(MP_E_INVALID, "NULL argument");
  if (P->precision != MP_FP64) return fail(MP_E_INVALID, "FP64 plans only");
  hipLaunchKernelGGL((k_rrm_points<double>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, P->stream,
                     long(n), static_cast<const uint8_t*>(phase), P->params,
                     static_cast<const double*>(e), static_cast<const double*>(g),
                     static_cast<const double*>(e_n), static_cast<const double*>(g_n),
                     static_cast<const double*>(t_n), static_cast<const double*>(m_n),
                     static_cast<const double*>(p_n), static_cast<const double*>(q_n),
                     static_cast<double*>(t), static_cast<double*>(m), static_cast<double*>(p),
                     static_cast<double*>(q));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

}  // extern "C"
