// Host side of the micropolar FFT solver: plan, workspace layout, Alg. 2
// step loop and the C ABI declared in include/mp.h.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace mp;

namespace mp {

// kernels of the single-RVE step loop (the batch runs the same device
// functions from its own kernels)
// block j reduces partial row j: error rows (avg = 0, rows 0..29) or
// step-average rows (avg = 1, rows 0..39)
__global__ void __launch_bounds__(256) k_rows(const double* partials, int nblk, int avg, double* tot,
                                              const Ctl* ctl) {
  if (ctl && ctl->done) return;
  __shared__ double red[4];
  const int j = blockIdx.x;
  const double v = row_reduce(glob(partials) + (long)j * nblk, nblk, !avg && err_row_is_max(j), red);
  if (threadIdx.x == 0) tot[j] = v;
}

__global__ void k_err_final(const double* tot, long nvox, Ctl* ctl, ErrMacro mac) {
  if (ctl->done || threadIdx.x != 0) return;
  err_finalize(tot, nvox, ctl, mac.v);
}

__global__ void k_ctl_reset(Ctl* ctl, int fixed, int max_iter, double tol, int norm) {
  ctl_reset(ctl, fixed, max_iter, tol, norm);
}

// Small cells (axes of 4 or 8, at most 128 voxels; FP64, isotropic
// reference medium, computed Green operator, basic scheme): the opening of a
// load step and its loop iterations in one block, up to max_loop iterations
// or until the control ends the step.  At these sizes each of the loop
// kernels is a few blocks and the loop runs at the GPU's per-kernel latency;
// here one launch runs the step.
// The half spectrum stays in LDS through the y and z passes; every pass
// takes the per-tile kernels' arithmetic (the same transforms per pencil,
// green_freq, xpass_tile, row_reduce's result through row_reduce_wave,
// err_finalize), so the iterates equal theirs bit for bit.  The control
// block is held in LDS across iterations (thread 0 updates it, a barrier
// publishes it) and written back at the end.  Within the block, a barrier
// orders the global writes of one pass before the reads of the next.
template <int N0, int L1, int L2>
struct SmallShape {
  using X = XShape<double, N0>;
  static constexpr int NTHR = 256;
  static constexpr int NH = N0 / 2;
  static constexpr int NB = NH * 18;        // one (kz, ky) run of kx and components
  static constexpr int PLANE = L1 * NB;     // one kz plane
  static constexpr int NS = L2 * PLANE;     // the half spectrum
  static constexpr int NXB = X::NPK * N0;   // one x-pass pencil buffer
  static constexpr size_t LDS =
      size_t(NS + 2 * NXB + N0 + L1 + L2) * sizeof(cx<double>) + size_t(NTHR / 64) * kRed * sizeof(double);
  static_assert(X::NTHR == NTHR, "x pass of 256 threads");
  static_assert(LDS <= 160 * 1024, "half spectrum and x buffers within 160 KB of LDS");
};

// The step's opening (open = 1, the step's first launch) runs in the same
// block first, as the per-kernel loop runs it before its loop kernels: the
// control reset, the TRANS x pass (commit of the previous step when
// xa.commit, first iterate of this one) and, after a commit, the step
// averages into tot_avg (k_rows' values, through row_reduce_wave).
struct SmallOpen {
  int open;
  int fixed, max_iter, norm;
  double tol;
  double* tot_avg;   // kNAvg step averages (sums) of the committed step
};

template <int N0, int L1, int L2>
__global__ void __launch_bounds__(256) k_small_loop(XArgs<double> xa, AxisArgs<double> az,
                                                    const cx<double>* twy_g, Ctl* ctl, ErrMacro em,
                                                    int ntiles, int max_loop, SmallOpen so) {
  using Q = SmallShape<N0, L1, L2>;
  constexpr int NTHR = Q::NTHR, NH = Q::NH, NB = Q::NB, PLANE = Q::PLANE, NS = Q::NS;
  extern __shared__ unsigned char smem_raw[];
  cx<double>* const spec = reinterpret_cast<cx<double>*>(smem_raw);
  cx<double>* const lds = spec + NS;
  cx<double>* const lds2 = lds + Q::NXB;
  cx<double>* const twx = lds2 + Q::NXB;
  cx<double>* const twy = twx + N0;
  cx<double>* const twz = twy + L1;
  double(*const red)[kRed] = reinterpret_cast<double(*)[kRed]>(twz + L2);
  __shared__ Ctl c;
  __shared__ double tot[kNPart];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  load_twiddles<double, N0, NTHR>(twx, glob(xa.tw), tid);
  load_twiddles<double, L1, NTHR>(twy, glob(twy_g), tid);
  load_twiddles<double, L2, NTHR>(twz, glob(az.tw), tid);
  if (tid == 0) {
    if (so.open)
      ctl_reset(&c, so.fixed, so.max_iter, so.tol, so.norm);
    else
      c = *ctl;
  }
  __syncthreads();
  MP_GLOBAL cx<double>* const S = glob(xa.S);
  const MP_GLOBAL double* const partials = glob(xa.partials);
  if (so.open) {
    for (int t = 0; t < ntiles; ++t) {
      xpass_tile<double, X_TRANS, N0>(xa, t, 0, ntiles, lds, lds2, red, twx, tid, false, false, nullptr);
      __syncthreads();
    }
    if (xa.commit) {
      constexpr int RPW = (kNAvg + 3) / 4;
      double x[RPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int j = wv + 4 * r;
        x[r] = (j < kNAvg && lane < ntiles) ? partials[long(j) * ntiles + lane] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int j = wv + 4 * r;
        if (j < kNAvg) {
          const double v = row_reduce_wave(x[r], lane, ntiles, false);
          if (lane == 0) glob(so.tot_avg)[j] = v;
        }
      }
      __syncthreads();
    }
  }
  for (int k = 0; k < max_loop && !c.done; ++k) {
    // y forward, z forward + Green operator + z inverse, y inverse
    for (int w = tid; w < NS; w += NTHR) spec[w] = gload(S + w);
    __syncthreads();
    for (int kz = 0; kz < L2; ++kz)
      fft_ct<double, false, L1, 1, NB, NB, 1, true, NTHR>(spec + kz * PLANE, twy, tid);
    fft_ct<double, false, L2, 1, PLANE, PLANE, 1, true, NTHR>(spec, twz, tid);
    for (int f = tid; f < L2 * L1 * NH; f += NTHR) {
      const int kx = f % NH, ky = (f / NH) % L1, kz = f / (NH * L1);
      green_freq<double, G_CLOSED>(az, kx, ky, kz, spec + (kz * L1 + ky) * NB + kx * 18);
    }
    __syncthreads();
    fft_ct<double, true, L2, 1, PLANE, PLANE, 1, true, NTHR>(spec, twz, tid);
    for (int kz = 0; kz < L2; ++kz)
      fft_ct<double, true, L1, 1, NB, NB, 1, true, NTHR>(spec + kz * PLANE, twy, tid);
    for (int w = tid; w < NS; w += NTHR) gstore(S + w, spec[w]);
    __syncthreads();
    // x pass ITER, tile by tile
    for (int t = 0; t < ntiles; ++t) {
      xpass_tile<double, X_ITER, N0>(xa, t, 0, ntiles, lds, lds2, red, twx, tid, false, false, nullptr);
      __syncthreads();
    }
    // error rows (wave wv takes rows wv, wv + 4, ...), then the measure
    constexpr int RPW = (kNPart + 3) / 4;
    double x[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = wv + 4 * r;
      x[r] = (j < kNPart && lane < ntiles) ? partials[long(j) * ntiles + lane] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = wv + 4 * r;
      if (j < kNPart) {
        const double v = row_reduce_wave(x[r], lane, ntiles, err_row_is_max(j));
        if (lane == 0) tot[j] = v;
      }
    }
    __syncthreads();
    if (tid == 0) err_finalize(tot, xa.nvox, &c, em.v);
    __syncthreads();
  }
  if (tid == 0) *ctl = c;
}

// FFT twiddle tables exp(-2 pi i m / n) of the three axes, one after the
// other (n0, then n1, then n2 entries), for the allocation-free spectral step
__global__ void k_twiddles(cx<double>* tw, int n0, int n1, int n2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0 + n1 + n2) return;
  const int n = i < n0 ? n0 : i < n0 + n1 ? n1 : n2;
  const int m = i < n0 ? i : i < n0 + n1 ? i - n0 : i - n0 - n1;
  double sn, cs;
  sincospi(-2.0 * double(m) / double(n), &sn, &cs);
  tw[i] = cx<double>{cs, sn};
}

}  // namespace mp

namespace {

constexpr int kProfEv = 6;     // boundaries around the 5 loop kernels of one iteration
constexpr int kRecord = 47;    // step record: 40 averages, err, iters, 4 err parts, reserved (0)

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
  double *pq, *out_pq, *partials, *tot;
  uint8_t* phase;
  PhaseC* params;
  void* tw0;      // cx<T>, n0 + n1 + n2 entries
  const void* eig;   // optional eigenstress (T, 18 n, caller-owned)
  const double* aniso;   // Eq. 5 row matrices, [record][level][81]
  const double* refan;   // general reference medium: its row matrices, or null
  const double* gsym;    // and its symbol coefficients [21][10], or null
  void* gtab;            // stored Green operator (T, [ky][kx][21][kz]), or null
  Ctl* ctl;
  Ctl* ctl_host;
  double* tot_host;   // pinned, kNAvg entries
  RefC ref;
  double tol;
  int max_iter, norm, fixed;
  bool al;        // augmented-Lagrangian iterations (MP_SCHEME_AL)
  double relax;   // their over-relaxation
  int n_phases;
  int steps;
  bool failed;            // a step diverged: no further steps
  double t_prev, t_cur;   // times of the last two committed states
  std::vector<std::vector<double>> resp_hist;
  // optional per-kernel timing of loop iterations (hipEvents on the plan's stream)
  int prof;   // 0 off, 1 every loop kernel, 2 the x pass only
  std::vector<hipEvent_t> ev;
  double prof_ms[8];
  long prof_n[8];
};

namespace {

// ---------------------------------------------------------------------------
// the one-block loop of small cells (k_small_loop)
// ---------------------------------------------------------------------------
#define MP_SMALL(X) X(4, 4, 4) X(4, 4, 8) X(4, 8, 4) X(8, 4, 4)

// the plan's loop iterations run in k_small_loop: FP64, a 4^3 cell or one
// axis of 8 and two of 4 (at most 128 voxels: one block runs an iteration of
// a 4^3 cell in 17 us against about 29 us for the six kernels, but one of
// an 8^3 cell in 65 us, its four x tiles one after another), an isotropic
// reference medium with the computed Green operator, Eq. 6 phases only, the
// basic scheme, and no per-kernel timing (which needs the kernels apart)
bool small_loop(const mp_plan_s* P) {
  const Geometry& g = P->g;
  auto ok = [](int n) { return n == 4 || n == 8; };
  return P->precision == MP_FP64 && ok(g.n0) && ok(g.n1) && ok(g.n2) && g.nvox <= 128 && g.n_aniso == 0 &&
         !g.ref_tensor && !P->gtab && !P->gsym && !P->refan && !P->al && P->prof == 0;
}

hipError_t prepare_small() {
  hipError_t e = hipSuccess;
#define MP_CASE(A, B, C)                                                                              \
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_loop<A, B, C>),                  \
                               hipFuncAttributeMaxDynamicSharedMemorySize,                            \
                               int(SmallShape<A, B, C>::LDS))) != hipSuccess)                          \
    return e;
  MP_SMALL(MP_CASE)
#undef MP_CASE
  return e;
}

template <int N0, int L1, int L2>
void launch_small_t(hipStream_t s, const XArgs<double>& xa, const AxisArgs<double>& az, const cx<double>* twy,
                    Ctl* ctl, const ErrMacro& em, int ntiles, int max_loop, const SmallOpen& so) {
  using Q = SmallShape<N0, L1, L2>;
  hipLaunchKernelGGL((k_small_loop<N0, L1, L2>), dim3(1), dim3(Q::NTHR), Q::LDS, s, xa, az, twy, ctl, em, ntiles,
                     max_loop, so);
}

void launch_small(int n0, int n1, int n2, hipStream_t s, const XArgs<double>& xa, const AxisArgs<double>& az,
                  const cx<double>* twy, Ctl* ctl, const ErrMacro& em, int ntiles, int max_loop,
                  const SmallOpen& so) {
#define MP_CASE(A, B, C)                                                              \
  if (n0 == A && n1 == B && n2 == C) {                                                \
    launch_small_t<A, B, C>(s, xa, az, twy, ctl, em, ntiles, max_loop, so);           \
    return;                                                                           \
  }
  MP_SMALL(MP_CASE)
#undef MP_CASE
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

  static AxisArgs<T> yargs(mp_plan P, cx<T>* S) {
    const Geometry& g = P->g;
    AxisArgs<T> a{};
    a.S = S;
    a.ostride = long(g.n1) * g.nh * 18;   // one kz plane
    a.pstride = long(g.nh) * 18;          // next ky
    a.tw = tw(P, 1);
    return a;
  }
  static AxisArgs<T> zargs(mp_plan P, cx<T>* S) {
    const Geometry& g = P->g;
    AxisArgs<T> a{};
    a.S = S;
    a.ostride = long(g.nh) * 18;          // next ky
    a.pstride = long(g.n1) * g.nh * 18;   // next kz
    a.tw = tw(P, 2);
    a.n0 = g.n0; a.n1 = g.n1; a.n2 = g.n2;
    a.h = P->h;
    a.scale = 1.0 / double(g.nvox);
    a.ref = P->ref;
    a.gsym = P->gsym;
    a.gtab = static_cast<const T*>(P->gtab);
    return a;
  }

  // y fwd, z fwd + Green + z inv, y inv (ev: optional events before each
  // kernel and after the last)
  static void spectral(mp_plan P, cx<T>* S, const Ctl* ctl, hipEvent_t* ev) {
    const Geometry& g = P->g;
    auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], P->stream); };
    const AxisArgs<T> ay = yargs(P, S), az = zargs(P, S);
    mark(0);
    launch_axis<T, Y_FWD>(g.n1, g.txy, g.nh / g.txy, g.n2, P->stream, ay, ctl);
    mark(1);
    if (P->gtab) {
      // the stored Green operator, on the closed form's tile widths
      const int tx = sizeof(T) == 4 && g.n2 >= 96 ? 1 : g.txz;
      launch_axis<T, Z_GREEN_ST>(g.n2, tx, g.nh / tx, g.n1, P->stream, az, ctl);
    } else if (P->gsym) {
      // FP64: one-wide tiles, whose kernels hold the per-frequency
      // factorisation without spilling (0.149 against 0.162 ms at 128^3)
      const int tx = sizeof(T) == 8 ? 1 : g.txz;
      launch_axis<T, Z_GREEN_AN>(g.n2, tx, g.nh / tx, g.n1, P->stream, az, ctl);
    } else {
      // FP32 from 96 points on: one-wide tiles (0.072 against 0.076 ms at
      // 128^3; the batch autotuner picks the same width for these classes)
      const int tx = sizeof(T) == 4 && g.n2 >= 96 ? 1 : g.txz;
      launch_axis<T, Z_GREEN>(g.n2, tx, g.nh / tx, g.n1, P->stream, az, ctl);
    }
    mark(2);
    launch_axis<T, Y_INV>(g.n1, g.txy, g.nh / g.txy, g.n2, P->stream, ay, ctl);
    mark(3);
  }

  static XArgs<T> xargs(mp_plan P) {
    const Geometry& g = P->g;
    XArgs<T> a{};
    a.nrows = g.nrows;
    a.tw = tw(P, 0);
    a.S = S(P);
    a.nvox = g.nvox;
    a.E = static_cast<double*>(P->E);
    a.Eprev = static_cast<double*>(P->Eprev);
    a.base = static_cast<T*>(P->base);
    a.pq = P->pq;
    a.out_tm = static_cast<T*>(P->out_tm);
    a.out_pq = P->out_pq;
    a.phase = P->phase;
    a.params = P->params;
    a.partials = P->partials;
    a.ref = P->ref;
    a.eig = static_cast<const T*>(P->eig);
    a.aniso = P->aniso;
    a.n_aniso = g.n_aniso;
    a.refan = P->refan;
    a.relax = P->relax;
    return a;
  }

  static hipError_t prepare() {
    hipError_t e;
    const int sizes[] = {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    for (int L : sizes) {
      if ((e = allow_lds<T, Y_FWD>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Y_INV>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_GREEN>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_GREEN_AN>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_GREEN_ST>(L)) != hipSuccess) return e;
      if ((e = allow_lds<T, Z_FWD>(L)) != hipSuccess) return e;
    }
    if constexpr (sizeof(T) == sizeof(double))
      if ((e = prepare_small()) != hipSuccess) return e;
    return hipSuccess;
  }

  static mp_status solve(mp_plan P, int32_t n_steps, const double* times, const double* E,
                         const double* Gam, int32_t* iters);
  static mp_status record_queue(mp_plan P);
  static void record_take(mp_plan P, std::vector<double>& rec);
  static mp_status record(mp_plan P, std::vector<double>& rec);
};

// Step averages of the committed state (rows of a TRANS x pass with
// commit set): reduce them and queue their copy to the host.  The loop
// kernels that follow on the stream overwrite the reduced rows only after
// the copy, so the record is taken at the next synchronisation.
template <class T>
mp_status Eng<T>::record_queue(mp_plan P) {
  const Geometry& g = P->g;
  hipLaunchKernelGGL(k_rows, dim3(kNAvg), dim3(256), 0, P->stream, P->partials, g.xblocks, 1, P->tot,
                     nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(P->tot_host, P->tot, kNAvg * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  return MP_OK;
}

// after the stream is synchronised: append the step record
template <class T>
void Eng<T>::record_take(mp_plan P, std::vector<double>& rec) {
  for (int j = 0; j < kNAvg; ++j) rec[j] = P->tot_host[j] / double(P->g.nvox);
  P->resp_hist.push_back(rec);
  P->steps += 1;
}

template <class T>
mp_status Eng<T>::record(mp_plan P, std::vector<double>& rec) {
  mp_status r = record_queue(P);
  if (r != MP_OK) return r;
  HIP_TRY(hipStreamSynchronize(P->stream));
  record_take(P, rec);
  return MP_OK;
}

template <class T>
mp_status Eng<T>::solve(mp_plan P, int32_t n_steps, const double* times, const double* E,
                        const double* Gam, int32_t* iters) {
  const Geometry& g = P->g;
  if (P->steps == 0) P->t_prev = P->t_cur = times[0];
  XArgs<T> xa = xargs(P);
  const bool small = small_loop(P);
  // the converged state of the previous step is committed by the x pass that
  // opens the next step (or by a commit-only pass after the last one)
  std::vector<double> rec(kRecord, 0.0);
  bool pending = false;
  mp_status st = MP_OK;
  std::string msg;
  for (int s = 1; s <= n_steps; ++s) {
    for (int c = 0; c < 9; ++c) {
      xa.mac[c] = E[(s - 1) * 9 + c];
      xa.mac[9 + c] = Gam[(s - 1) * 9 + c];
    }
    xa.first = P->steps == 0 && !pending;
    // Alg. 2 linear extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
    xa.r = xa.first ? 0.0 : (times[s] - P->t_cur) / (P->t_cur - P->t_prev);
    xa.commit = pending;
    xa.init = 1;
    P->ctl_host->iters = 0;
    P->ctl_host->done = 0;
    // the previous step's record, taken at the loop's first synchronisation
    const bool take_rec = pending;
    bool take = false;
    if (!small) {
      hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, P->stream, P->ctl, P->fixed, P->max_iter,
                         P->tol, P->norm);
      // commit of the previous step, first iterate of this one (extrapolated
      // or uniform), its return map and polarization
      launch_x<T, X_TRANS>(g.n0, g.xblocks, P->stream, xa, nullptr, g.n_aniso > 0 || g.ref_tensor);
      if (pending) {
        mp_status r = record_queue(P);
        if (r != MP_OK) return r;
        take = true;
      }
    }
    // (a small cell opens the step in its first loop launch below)
    pending = false;
    ErrMacro em;
    for (int c = 0; c < 18; ++c) em.v[c] = xa.mac[c];
    // the one-block loop of a small cell runs until the control ends the
    // step, in launches of at most kSmallLoop iterations (a step of a
    // typical count is one launch; no launch runs for long, about 70 ms at
    // 4^3).  Otherwise batches of 2, 4, 8, ... 64 iterations (kernels
    // queued past the end of the step return at once)
    constexpr long kSmallLoop = 4096;
    int batch = small ? int(std::min(long(std::max(P->max_iter, P->fixed)) + 1, kSmallLoop)) : 2;
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
      bool fused = false;
      if constexpr (sizeof(T) == sizeof(double)) {
        if (small) {
          SmallOpen so{queued == batch ? 1 : 0, P->fixed, P->max_iter, P->norm, P->tol, P->tot};
          launch_small(g.n0, g.n1, g.n2, P->stream, xa, zargs(P, S(P)), tw(P, 1), P->ctl, em, g.xblocks, batch,
                       so);
          if (so.open && take_rec) {
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(P->tot_host, P->tot, kNAvg * sizeof(double), hipMemcpyDeviceToHost,
                                   P->stream));
            take = true;
          }
          fused = true;
        }
      }
      for (int k = 0; k < batch && !fused; ++k) {
        // profiling: events between all loop kernels (mode 1) or around the
        // x pass only (mode 2, two event records per iteration)
        hipEvent_t* ev = P->prof ? &P->ev[size_t(k) * kProfEv] : nullptr;
        spectral(P, S(P), P->ctl, P->prof == 1 ? ev : nullptr);
        if (P->prof == 2) HIP_TRY(hipEventRecord(ev[3], P->stream));
        launch_x<T, X_ITER>(g.n0, g.xblocks, P->stream, xa, P->ctl, g.n_aniso > 0 || g.ref_tensor, P->al);
        if (ev) HIP_TRY(hipEventRecord(ev[4], P->stream));
        hipLaunchKernelGGL(k_rows, dim3(kNPart), dim3(256), 0, P->stream, P->partials, g.xblocks, 0,
                           P->tot, P->ctl);
        hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, P->stream, P->tot, g.nvox, P->ctl, em);
        if (P->prof == 1) HIP_TRY(hipEventRecord(ev[5], P->stream));
      }
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(P->ctl_host, P->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
      HIP_TRY(hipStreamSynchronize(P->stream));
      if (take) {
        record_take(P, rec);
        take = false;
      }
      if (P->prof) {
        // only iterations that really ran (later ones returned at once)
        const int ran = std::min(batch, P->ctl_host->iters - it0);
        for (int k = 0; k < ran; ++k)
          for (int j = 0; j < kProfEv - 1; ++j) {
            if (P->prof == 2 && j != 3) continue;
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, P->ev[size_t(k) * kProfEv + j],
                                        P->ev[size_t(k) * kProfEv + j + 1]));
            P->prof_ms[j] += ms;
            P->prof_n[j] += 1;
          }
      }
      if (P->ctl_host->done) break;
      if (!small) batch = std::min(batch * 2, 64);
    }
    const Ctl c = *P->ctl_host;
    if (iters) iters[s - 1] = c.iters;
    if (c.done == 3) {
      // a diverged iterate is no converged state: the step is not committed,
      // and the plan takes no further steps
      P->failed = true;
      st = MP_E_DIVERGED;
      msg = "step " + std::to_string(P->steps + 1) + " diverged (not committed)";
      break;
    }
    std::fill(rec.begin(), rec.end(), 0.0);
    rec[40] = c.err;
    rec[41] = c.iters;
    for (int f = 0; f < 4; ++f) rec[42 + f] = c.err_parts[f];
    rec[46] = 0.0;
    pending = true;
    P->t_prev = P->t_cur;
    P->t_cur = times[s];
    if (c.done == 2) {
      st = MP_E_NOT_CONVERGED;
      msg = "step " + std::to_string(P->steps + 1) + " hit max_iter (committed)";
      break;
    }
  }
  if (pending) {
    // commit only: the last step of this call (or the failed one)
    xa.commit = 1;
    xa.init = 0;
    launch_x<T, X_TRANS>(g.n0, g.xblocks, P->stream, xa, nullptr, g.n_aniso > 0 || g.ref_tensor);
    mp_status r = record(P, rec);
    if (r != MP_OK) return r;
  }
  if (st != MP_OK) return fail(st, msg);
  return MP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free spectral step (mp_green_apply_noalloc): the
// half spectra and the twiddle tables live in this file-scope device array,
// of which every device holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel: on the host it is a
// stand-in, not a device address.  It uses the address hipGetSymbolAddress
// gives for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(48) << 20;   // 48 MiB: an FP64 64^3 grid fits
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices];   // scratch's device address per device (null: not set up)

// Device address of `scratch` on the current device; the first call on a
// device also raises the axis kernels' LDS limits there.
mp_status scratch_address(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MP_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(MP_E_DEVICE, "hipGetSymbolAddress gave a null scratch address");
    HIP_TRY(Eng<double>::prepare());
    g_scratch_dev[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_dev[dev];
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
  P->eig = nullptr;
  P->aniso = reinterpret_cast<const double*>(wsp + L.aniso);
  P->refan = nullptr;
  P->gsym = nullptr;
  P->gtab = g.green_stored ? static_cast<void*>(wsp + L.gtab) : nullptr;
  P->partials = reinterpret_cast<double*>(wsp + L.partials);
  P->ctl = reinterpret_cast<Ctl*>(wsp + L.ctl);
  P->tot = reinterpret_cast<double*>(wsp + L.tot);
  P->tol = prob->tol;
  P->max_iter = prob->max_iter;
  P->norm = prob->err_norm;
  P->fixed = 0;
  P->al = prob->scheme == MP_SCHEME_AL;
  P->relax = P->al ? prob->relax : 1.0;
  P->prof = 0;
  for (int j = 0; j < 8; ++j) { P->prof_ms[j] = 0.0; P->prof_n[j] = 0; }
  P->n_phases = prob->n_phases;
  P->steps = 0;
  P->failed = false;
  P->t_prev = P->t_cur = 0.0;

  // reference medium (Alg. 2: A0 = <A>, B0 = <B>); phase mean by default
  {
    const mp_status rs = reference_medium(prob, g.nvox, &P->ref);
    if (rs != MP_OK) {
      delete P;
      return rs;
    }
  }

  std::vector<PhaseC> pc(256);
  for (int i = 0; i < prob->n_phases; ++i) pc[i] = derive(prob->phases[i]);
  std::vector<double> arows(aniso_words(g), 0.0);
  for (int j = 0; j < g.n_aniso; ++j) {
    aniso_rows(prob->aniso[j], &arows[size_t(j) * 162]);
    pc[prob->aniso[j].phase].t.aid = double(j);
  }
  if (g.ref_tensor) {
    // general reference medium: its row matrices after the phases' records,
    // then the coefficients of its Fourier symbol
    mp_aniso r;
    const mp_status rs = reference_tensors(prob, g.nvox, &r);
    if (rs != MP_OK) {
      delete P;
      return rs;
    }
    aniso_rows(r, &arows[size_t(g.n_aniso) * 162]);
    green_symbol(r, &arows[sym_offset(g)]);
    P->refan = P->aniso + size_t(g.n_aniso) * 162;
    P->gsym = P->aniso + sym_offset(g);
  } else if (g.green_stored) {
    // the symbol of the isotropic reference, from its Eq. 6 tensors, for
    // the stored Green operator
    mp_phase c{};
    c.lambda = P->ref.lam; c.mu = P->ref.mu; c.kappa = P->ref.kap;
    c.alpha = P->ref.alp; c.beta = P->ref.bet; c.gamma = P->ref.gam;
    mp_aniso r{};
    iso_tensors(c, r.A, r.B);
    green_symbol(r, &arows[sym_offset(g)]);
  }
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

  auto cleanup = [&](mp_status st) {
    if (P->ctl_host) (void)hipHostFree(P->ctl_host);
    if (P->tot_host) (void)hipHostFree(P->tot_host);
    delete P;
    return st;
  };
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
  CREATE_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->tot_host), kNAvg * sizeof(double)));
  CREATE_TRY(hipMemsetAsync(wsp, 0, L.total, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->phase, prob->phase, g.nvox, hipMemcpyHostToDevice, P->stream));
  CREATE_TRY(hipMemcpyAsync(P->params, pc.data(), pc.size() * sizeof(PhaseC), hipMemcpyHostToDevice,
                            P->stream));
  CREATE_TRY(hipMemcpyAsync(wsp + L.aniso, arows.data(), arows.size() * sizeof(double),
                            hipMemcpyHostToDevice, P->stream));
  if (mixed) {
    CREATE_TRY(hipMemcpyAsync(P->tw0, twf.data(), twf.size() * sizeof(cx<float>),
                              hipMemcpyHostToDevice, P->stream));
  } else {
    CREATE_TRY(hipMemcpyAsync(P->tw0, tw.data(), tw.size() * sizeof(cx<double>),
                              hipMemcpyHostToDevice, P->stream));
  }
  if (P->gtab) {
    // the stored Green operator (Sec. 2.4): once, from the symbol coefficients
    const long nf = g.nspec;
    const int blocks = int(std::min<long>((nf + 255) / 256, 4096));
    const double* coef = P->aniso + sym_offset(g);
    if (mixed)
      hipLaunchKernelGGL(k_green_table<float>, dim3(blocks), dim3(256), 0, P->stream, coef, g.n0, g.n1, g.n2,
                         P->h, static_cast<float*>(P->gtab));
    else
      hipLaunchKernelGGL(k_green_table<double>, dim3(blocks), dim3(256), 0, P->stream, coef, g.n0, g.n1,
                         g.n2, P->h, static_cast<double*>(P->gtab));
    CREATE_TRY(hipGetLastError());
  }
  CREATE_TRY(hipStreamSynchronize(P->stream));
#undef CREATE_TRY
  *out = P;
  return MP_OK;
}

void mp_plan_destroy(mp_plan P) {
  if (!P) return;
  if (P->ctl_host) (void)hipHostFree(P->ctl_host);
  if (P->tot_host) (void)hipHostFree(P->tot_host);
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  delete P;
}

mp_status mp_profile(mp_plan P, int32_t mode) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  if (mode < 0 || mode > 2) return fail(MP_E_INVALID, "profile mode must be 0, 1 or 2");
  P->prof = mode;
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

mp_status mp_set_eigenstress(mp_plan P, const void* dev_eig) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  P->eig = dev_eig;
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
  if (P->failed) return fail(MP_E_STATE, "a step of this plan diverged; it takes no further steps");
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

mp_status mp_get_fields(mp_plan P, uint32_t mask, void* const* dst, int32_t dst_is_device) {
  if (!P) return fail(MP_E_INVALID, "plan is NULL");
  const size_t w = P->precision == MP_MIXED ? sizeof(float) : sizeof(double);
  return copy_fields(static_cast<const unsigned char*>(P->E), static_cast<const unsigned char*>(P->out_tm),
                     reinterpret_cast<const unsigned char*>(P->out_pq), P->g.nvox, w, mask, dst,
                     dst_is_device, P->stream);
}

mp_status mp_spectrum_forward(mp_plan P, const void* dev_in, void* dev_out) {
  if (!P || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  if (P->precision != MP_FP64) return fail(MP_E_INVALID, "FP64 plans only");
  using E8 = Eng<double>;
  const Geometry& g = P->g;
  XArgs<double> xa = E8::xargs(P);
  xa.fin = static_cast<const double*>(dev_in);
  cx<double>* S = static_cast<cx<double>*>(dev_out);
  xa.S = S;
  launch_x<double, X_FWD_ONLY>(g.n0, g.xblocks, P->stream, xa, nullptr);
  launch_axis<double, Y_FWD>(g.n1, g.txy, g.nh / g.txy, g.n2, P->stream, E8::yargs(P, S),
                             nullptr);
  launch_axis<double, Z_FWD>(g.n2, g.txz, g.nh / g.txz, g.n1, P->stream, E8::zargs(P, S),
                             nullptr);
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
  xa.fin = static_cast<const double*>(dev_in);
  launch_x<double, X_FWD_ONLY>(g.n0, g.xblocks, P->stream, xa, nullptr);
  E8::spectral(P, E8::S(P), nullptr, nullptr);
  xa.fout = static_cast<double*>(dev_out);
  launch_x<double, X_INV_ONLY>(g.n0, g.xblocks, P->stream, xa, nullptr);
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
  if (P->g.n_aniso > 0) return fail(MP_E_INVALID, "plans with Eq. 5 phases are not supported here");
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

mp_status mp_green_apply_noalloc(const int32_t n[3], double h, const double ref[6], const void* dev_in,
                                 void* dev_out, void* hip_stream) {
  if (!n || !ref || !dev_in || !dev_out) return fail(MP_E_INVALID, "NULL argument");
  for (int i = 0; i < 3; ++i)
    if (!supported(n[i]))
      return fail(MP_E_INVALID, "grid size n[" + std::to_string(i) + "] = " + std::to_string(n[i]) +
                                    " unsupported (4 6 8 12 16 24 32 48 64 96 128 192 256)");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(MP_E_INVALID, "h must be > 0");
  const RefC r{ref[0], ref[1], ref[2], ref[3], ref[4], ref[5]};
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(ref[k])) return fail(MP_E_INVALID, "reference constants must be finite");
  if (!(r.lam + 2 * r.mu > 0) || !(r.mu > 0) || !(r.kap > 0) || !(r.gam > 0) || !(r.alp + r.bet + r.gam > 0))
    return fail(MP_E_INVALID, "reference medium is not positive definite");
  const Geometry g = grid_geometry(n[0], n[1], n[2]);
  const size_t spec = align256(size_t(18) * g.nspec * sizeof(cx<double>));
  const size_t need = spec + size_t(g.n0 + g.n1 + g.n2) * sizeof(cx<double>);
  if (need > kScratchBytes)
    return fail(MP_E_INVALID, "grid needs " + std::to_string(need) + " bytes of scratch; the limit is " +
                                  std::to_string(kScratchBytes) + " (48 MiB)");
  unsigned char* ptr = nullptr;
  const mp_status st = scratch_address(&ptr);
  if (st != MP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  cx<double>* S = reinterpret_cast<cx<double>*>(ptr);
  cx<double>* tw = reinterpret_cast<cx<double>*>(ptr + spec);
  const int ntw = g.n0 + g.n1 + g.n2;
  hipLaunchKernelGGL(k_twiddles, dim3(unsigned((ntw + 255) / 256)), dim3(256), 0, s, tw, g.n0, g.n1, g.n2);
  XArgs<double> xa{};
  xa.nrows = g.nrows;
  xa.tw = tw;
  xa.S = S;
  xa.nvox = g.nvox;
  xa.fin = static_cast<const double*>(dev_in);
  xa.fout = static_cast<double*>(dev_out);
  AxisArgs<double> ay{};
  ay.S = S;
  ay.ostride = long(g.n1) * g.nh * 18;
  ay.pstride = long(g.nh) * 18;
  ay.tw = tw + g.n0;
  AxisArgs<double> az{};
  az.S = S;
  az.ostride = long(g.nh) * 18;
  az.pstride = long(g.n1) * g.nh * 18;
  az.tw = tw + g.n0 + g.n1;
  az.n0 = g.n0;
  az.n1 = g.n1;
  az.n2 = g.n2;
  az.h = h;
  az.scale = 1.0 / double(g.nvox);
  az.ref = r;
  az.gsym = nullptr;
  // the kernels and tile widths of mp_green_apply on an FP64 plan
  launch_x<double, X_FWD_ONLY>(g.n0, g.xblocks, s, xa, nullptr);
  launch_axis<double, Y_FWD>(g.n1, g.txy, g.nh / g.txy, g.n2, s, ay, nullptr);
  launch_axis<double, Z_GREEN>(g.n2, g.txz, g.nh / g.txz, g.n1, s, az, nullptr);
  launch_axis<double, Y_INV>(g.n1, g.txy, g.nh / g.txy, g.n2, s, ay, nullptr);
  launch_x<double, X_INV_ONLY>(g.n0, g.xblocks, s, xa, nullptr);
  HIP_TRY(hipGetLastError());
  return MP_OK;
}

}  // extern "C"
