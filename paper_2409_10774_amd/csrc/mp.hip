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

// radix schedule (8s first, then 4, 2, 3): 4 bits per stage
bool radix_schedule(int n, uint32_t* sched, std::vector<int>* radices) {
  std::vector<int> r;
  int m = n;
  while (m % 8 == 0) { r.push_back(8); m /= 8; }
  while (m % 4 == 0) { r.push_back(4); m /= 4; }
  while (m % 2 == 0) { r.push_back(2); m /= 2; }
  while (m % 3 == 0) { r.push_back(3); m /= 3; }
  if (m != 1 || r.size() > 8) return false;
  uint32_t s = 0;
  for (size_t i = 0; i < r.size(); ++i) s |= uint32_t(r[i]) << (4 * i);
  *sched = s;
  if (radices) *radices = r;
  return true;
}

// every stage must fit kMaxPts points per thread
bool fits(int N, int nb, int nthr, const std::vector<int>& radices) {
  for (int R : radices) {
    const long total = long(N / R) * nb;
    const long per = (total + nthr - 1) / nthr;
    if (per * R > kMaxPts) return false;
  }
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t S, E, Eprev, base, pq, out_tm, out_pq, phase, params, tw, partials, ctl, tot, resp, total;
};

struct Geometry {
  int n0, n1, n2, nh;
  long nvox, nspec;
  int rows, xthreads, xblocks;
  int txy, txz;
  uint32_t s0, s1, s2;
  int commit_blocks;
};

}  // namespace

struct mp_plan_s {
  Geometry g;
  Layout L;
  double h;
  hipStream_t stream;
  unsigned char* ws;
  cx<double>* S;
  double *E, *Eprev, *base, *pq, *out_tm, *out_pq, *partials, *tot, *resp;
  uint8_t* phase;
  PhaseC* params;
  cx<double>* tw0;
  cx<double>* tw1;
  cx<double>* tw2;
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
  std::vector<hipEvent_t> ev;    // kProfEv events per queued iteration
  double prof_ms[8];
  long prof_n[8];
};

namespace {

mp_status validate(const mp_problem* p, Geometry* g) {
  if (!p) return fail(MP_E_INVALID, "problem is NULL");
  for (int i = 0; i < 3; ++i) {
    const int n = p->n[i];
    uint32_t s;
    if (n < 4 || n > 256 || (n & 1) || !radix_schedule(n, &s, nullptr))
      return fail(MP_E_INVALID, "grid size n[" + std::to_string(i) + "] = " + std::to_string(n) +
                                    " unsupported (even, 4..256, 2^a 3^b)");
  }
  if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(MP_E_INVALID, "h must be > 0");
  if (p->n_phases < 1 || p->n_phases > 256) return fail(MP_E_INVALID, "n_phases out of 1..256");
  if (!p->phase || !p->phases) return fail(MP_E_INVALID, "phase map / table is NULL");
  if (!(p->tol > 0.0)) return fail(MP_E_INVALID, "tol must be > 0");
  if (p->max_iter < 1) return fail(MP_E_INVALID, "max_iter must be >= 1");
  if (p->err_norm != MP_ERR_LOCAL && p->err_norm != MP_ERR_AVERAGE)
    return fail(MP_E_INVALID, "err_norm");
  if (p->precision != MP_FP64) return fail(MP_E_INVALID, "only MP_FP64 is built");
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
  std::vector<int> r0, r1, r2;
  radix_schedule(G.n0, &G.s0, &r0);
  radix_schedule(G.n1, &G.s1, &r1);
  radix_schedule(G.n2, &G.s2, &r2);
  // x pass: rows per block (a divisor of n1 n2), two lanes per voxel
  const long nrows = long(G.n1) * G.n2;
  int rows = std::max(1, 128 / G.n0);
  while (rows > 1 && nrows % rows) --rows;
  G.rows = rows;
  G.xthreads = 2 * ((rows * G.n0 + 63) / 64 * 64);
  if (G.xthreads > 512 || !fits(G.n0, 9 * rows, G.xthreads, r0))
    return fail(MP_E_INVALID, "x pass does not fit");
  G.xblocks = int(nrows / rows);
  // y / z passes: tile width TX | nh
  auto pick_tx = [&](int L, const std::vector<int>& rad) {
    for (int tx = 16; tx >= 1; tx >>= 1)
      if (G.nh % tx == 0 && fits(L, tx, 256, rad)) return tx;
    return 0;
  };
  G.txy = pick_tx(G.n1, r1);
  G.txz = pick_tx(G.n2, r2);
  if (!G.txy || !G.txz) return fail(MP_E_INVALID, "y/z pass does not fit");
  G.commit_blocks = int((nvox + 255) / 256);
  *g = G;
  return MP_OK;
}

Layout layout(const Geometry& g) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.S = take(18 * g.nspec * sizeof(cx<double>));
  L.E = take(18 * g.nvox * sizeof(double));
  L.Eprev = take(18 * g.nvox * sizeof(double));
  L.base = take(18 * g.nvox * sizeof(double));
  L.pq = take(2 * g.nvox * sizeof(double));
  L.out_tm = take(18 * g.nvox * sizeof(double));
  L.out_pq = take(2 * g.nvox * sizeof(double));
  L.phase = take(g.nvox);
  L.params = take(256 * sizeof(PhaseC));
  L.tw = take(size_t(g.n0 + g.n1 + g.n2) * sizeof(cx<double>));
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

void twiddles(int n, std::vector<cx<double>>* out) {
  for (int m = 0; m < n; ++m) {
    // exp(-2 pi i m / n), argument reduced to the first half-turn for accuracy
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * m / n;
    out->push_back(cx<double>{double(cosl(a)), double(sinl(a))});
  }
}

constexpr int kProfEv = 8;     // boundaries around the 7 kernels of one iteration

// enqueue the spectral part: y fwd, z fwd, Green, z inv, y inv
// (ev: optional array of 6 events recorded before each kernel and after the last)
void enqueue_spectral(mp_plan P, const Ctl* ctl, hipEvent_t* ev = nullptr) {
  const Geometry& g = P->g;
  AxisArgs<double> ay{P->S, g.nspec, long(g.n1) * g.nh, g.nh, g.n1, g.txy, g.s1, P->tw1, ctl};
  AxisArgs<double> az{P->S, g.nspec, g.nh, long(g.n1) * g.nh, g.n2, g.txz, g.s2, P->tw2, ctl};
  dim3 gy(g.nh / g.txy, g.n2, 18), gz(g.nh / g.txz, g.n1, 18);
  const size_t shy = size_t(g.n1) * g.txy * sizeof(cx<double>);
  const size_t shz = size_t(g.n2) * g.txz * sizeof(cx<double>);
  auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], P->stream); };
  mark(0);
  hipLaunchKernelGGL((k_axis<double, false>), gy, dim3(256), shy, P->stream, ay);
  mark(1);
  hipLaunchKernelGGL((k_axis<double, false>), gz, dim3(256), shz, P->stream, az);
  mark(2);
  GreenArgs<double> ga{P->S, g.nspec, g.n0, g.n1, g.n2, g.nh, P->h,
                       1.0 / double(g.nvox), P->ref, ctl};
  hipLaunchKernelGGL((k_green<double>), dim3(unsigned((g.nspec + 255) / 256)), dim3(256), 0,
                     P->stream, ga);
  mark(3);
  hipLaunchKernelGGL((k_axis<double, true>), gz, dim3(256), shz, P->stream, az);
  mark(4);
  hipLaunchKernelGGL((k_axis<double, true>), gy, dim3(256), shy, P->stream, ay);
  mark(5);
}

XArgs<double> xargs(mp_plan P) {
  const Geometry& g = P->g;
  XArgs<double> a{};
  a.n0 = g.n0; a.n1 = g.n1; a.n2 = g.n2; a.nh = g.nh; a.rows = g.rows;
  a.sched = g.s0; a.tw = P->tw0; a.S = P->S; a.nspec = g.nspec; a.nvox = g.nvox;
  a.E = P->E; a.Eprev = P->Eprev; a.base = P->base; a.pq = P->pq; a.phase = P->phase;
  a.params = P->params; a.partials = P->partials; a.ctl = P->ctl; a.ref = P->ref;
  return a;
}

size_t xshared(const Geometry& g) { return size_t(9) * g.rows * g.n0 * sizeof(cx<double>); }

}  // namespace

extern "C" {

const char* mp_last_error(void) { return g_err.c_str(); }
const char* mp_version(void) { return "mp 0.1 gfx950"; }

mp_status mp_plan_workspace_size(const mp_problem* prob, size_t* bytes) {
  Geometry g;
  mp_status s = validate(prob, &g);
  if (s != MP_OK) return s;
  if (!bytes) return fail(MP_E_INVALID, "bytes is NULL");
  *bytes = layout(g).total;
  return MP_OK;
}

mp_status mp_plan_create(const mp_problem* prob, void* dev_workspace, size_t bytes, void* hip_stream,
                         mp_plan* out) {
  Geometry g;
  mp_status s = validate(prob, &g);
  if (s != MP_OK) return s;
  if (!out) return fail(MP_E_INVALID, "out is NULL");
  Layout L = layout(g);
  if (!dev_workspace || bytes < L.total)
    return fail(MP_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255)
    return fail(MP_E_INVALID, "workspace must be 256-byte aligned");

  mp_plan P = new mp_plan_s();
  P->g = g;
  P->L = L;
  P->h = prob->h;
  P->stream = reinterpret_cast<hipStream_t>(hip_stream);
  unsigned char* w = static_cast<unsigned char*>(dev_workspace);
  P->ws = w;
  P->S = reinterpret_cast<cx<double>*>(w + L.S);
  P->E = reinterpret_cast<double*>(w + L.E);
  P->Eprev = reinterpret_cast<double*>(w + L.Eprev);
  P->base = reinterpret_cast<double*>(w + L.base);
  P->pq = reinterpret_cast<double*>(w + L.pq);
  P->out_tm = reinterpret_cast<double*>(w + L.out_tm);
  P->out_pq = reinterpret_cast<double*>(w + L.out_pq);
  P->phase = w + L.phase;
  P->params = reinterpret_cast<PhaseC*>(w + L.params);
  P->tw0 = reinterpret_cast<cx<double>*>(w + L.tw);
  P->tw1 = P->tw0 + g.n0;
  P->tw2 = P->tw1 + g.n1;
  P->partials = reinterpret_cast<double*>(w + L.partials);
  P->ctl = reinterpret_cast<Ctl*>(w + L.ctl);
  P->tot = reinterpret_cast<double*>(w + L.tot);
  P->resp = reinterpret_cast<double*>(w + L.resp);
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
  twiddles(g.n0, &tw);
  twiddles(g.n1, &tw);
  twiddles(g.n2, &tw);

  auto cleanup = [&](mp_status st) { delete P; return st; };
  hipError_t e;
#define CREATE_TRY(call)                                                                 \
  if ((e = (call)) != hipSuccess) {                                                      \
    g_err = std::string(#call) + ": " + hipGetErrorString(e);                            \
    return cleanup(MP_E_DEVICE);                                                         \
  }
  CREATE_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->ctl_host), sizeof(Ctl)));
  CREATE_TRY(hipMemsetAsync(w, 0, L.total, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->phase, prob->phase, g.nvox, hipMemcpyHostToDevice, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->params, pc.data(), pc.size() * sizeof(PhaseC), hipMemcpyHostToDevice,
                            P->stream));
  CREATE_TRY(hipMemcpyAsync(P->tw0, tw.data(), tw.size() * sizeof(cx<double>), hipMemcpyHostToDevice,
                            P->stream));
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
  for (int j = 0; j < n && j < 7; ++j) {
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
  if (P->steps == 0) P->t_prev = P->t_cur = times[0];
  const Geometry& g = P->g;
  for (int s = 1; s <= n_steps; ++s) {
    XArgs<double> xa = xargs(P);
    for (int c = 0; c < 9; ++c) {
      xa.mac[c] = E[(s - 1) * 9 + c];
      xa.mac[9 + c] = Gam[(s - 1) * 9 + c];
    }
    xa.first = P->steps == 0;
    // Alg. 2 linear extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
    xa.r = P->steps == 0 ? 0.0 : (times[s] - P->t_cur) / (P->t_cur - P->t_prev);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, P->stream, P->ctl, P->fixed, P->max_iter,
                       P->tol, P->norm);
    P->ctl_host->iters = 0;
    P->ctl_host->done = 0;
    // first iterate (extrapolated or uniform), its return map and polarization
    xa.ctl = nullptr;
    hipLaunchKernelGGL((k_xpass<double, X_INIT>), dim3(g.xblocks), dim3(g.xthreads), xshared(g),
                       P->stream, xa);
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
        enqueue_spectral(P, P->ctl, ev);
        hipLaunchKernelGGL((k_xpass<double, X_ITER>), dim3(g.xblocks), dim3(g.xthreads), xshared(g),
                           P->stream, xa);
        if (ev) HIP_TRY(hipEventRecord(ev[6], P->stream));
        hipLaunchKernelGGL(k_err_rows, dim3(kNPart), dim3(256), 0, P->stream, P->partials, g.xblocks,
                           P->tot, P->ctl);
        hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, P->stream, P->tot, g.nvox, P->ctl, em);
        if (ev) HIP_TRY(hipEventRecord(ev[7], P->stream));
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
            // kernel order: y fwd, z fwd, green, z inv, y inv, x pass, error reduce
            P->prof_ms[j] += ms;
            P->prof_n[j] += 1;
          }
      }
      if (P->ctl_host->done) break;
      batch = std::min(batch * 2, 64);
    }
    const Ctl c = *P->ctl_host;
    // commit
    CommitArgs<double> ca{g.nvox, P->E, P->base, P->pq, P->out_tm, P->out_pq, P->phase, P->params,
                          P->partials};
    hipLaunchKernelGGL((k_commit<double>), dim3(g.commit_blocks), dim3(256), 0, P->stream, ca);
    hipLaunchKernelGGL(k_avg_reduce, dim3(1), dim3(256), 0, P->stream, P->partials, g.commit_blocks,
                       g.nvox, P->resp);
    std::vector<double> r(42, 0.0);
    HIP_TRY(hipMemcpyAsync(r.data(), P->resp, kNAvg * sizeof(double), hipMemcpyDeviceToHost,
                           P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    r[40] = c.err;
    r[41] = c.iters;
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

mp_status mp_homogenized_response(mp_plan P, int32_t step, double out[42]) {
  if (!P || !out) return fail(MP_E_INVALID, "NULL argument");
  if (step < 1 || step > P->steps) return fail(MP_E_INVALID, "step out of range");
  std::memcpy(out, P->resp_hist[step - 1].data(), 42 * sizeof(double));
  return MP_OK;
}

mp_status mp_get_fields(mp_plan P, int32_t field, double* dst) {
  if (!P || !dst) return fail(MP_E_INVALID, "NULL argument");
  const long n = P->g.nvox;
  const double* src = nullptr;
  long count = 9 * n;
  switch (field) {
    case MP_FIELD_E: src = P->E; break;
    case MP_FIELD_GAMMA: src = P->E + 9 * n; break;
    case MP_FIELD_T: src = P->out_tm; break;
    case MP_FIELD_M: src = P->out_tm + 9 * n; break;
    case MP_FIELD_P: src = P->out_pq; count = n; break;
    case MP_FIELD_Q: src = P->out_pq + n; count = n; break;
    default: return fail(MP_E_INVALID, "unknown field");
  }
  HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

mp_status mp_spectrum_forward(mp_plan P, const void* dev_in, void* dev_out) {
  if (!P || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  const Geometry& g = P->g;
  XArgs<double> xa = xargs(P);
  xa.ctl = nullptr;
  xa.fin = static_cast<const double*>(dev_in);
  xa.S = static_cast<cx<double>*>(dev_out);
  hipLaunchKernelGGL((k_xpass<double, X_FWD_ONLY>), dim3(g.xblocks), dim3(g.xthreads), xshared(g),
                     P->stream, xa);
  cx<double>* S = static_cast<cx<double>*>(dev_out);
  AxisArgs<double> ay{S, g.nspec, long(g.n1) * g.nh, g.nh, g.n1, g.txy, g.s1, P->tw1, nullptr};
  AxisArgs<double> az{S, g.nspec, g.nh, long(g.n1) * g.nh, g.n2, g.txz, g.s2, P->tw2, nullptr};
  hipLaunchKernelGGL((k_axis<double, false>), dim3(g.nh / g.txy, g.n2, 18), dim3(256),
                     size_t(g.n1) * g.txy * sizeof(cx<double>), P->stream, ay);
  hipLaunchKernelGGL((k_axis<double, false>), dim3(g.nh / g.txz, g.n1, 18), dim3(256),
                     size_t(g.n2) * g.txz * sizeof(cx<double>), P->stream, az);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MP_OK;
}

mp_status mp_green_apply(mp_plan P, const void* dev_in, void* dev_out) {
  if (!P || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  const Geometry& g = P->g;
  XArgs<double> xa = xargs(P);
  xa.ctl = nullptr;
  xa.fin = static_cast<const double*>(dev_in);
  hipLaunchKernelGGL((k_xpass<double, X_FWD_ONLY>), dim3(g.xblocks), dim3(g.xthreads), xshared(g),
                     P->stream, xa);
  enqueue_spectral(P, nullptr);
  xa.fout = static_cast<double*>(dev_out);
  hipLaunchKernelGGL((k_xpass<double, X_INV_ONLY>), dim3(g.xblocks), dim3(g.xthreads), xshared(g),
                     P->stream, xa);
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
