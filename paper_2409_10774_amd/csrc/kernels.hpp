// Kernels of one fixed-point iteration of the micropolar basic scheme (Alg. 2)
// and of the step control around it.
//
// Field layout in HBM (SoA, x fastest, voxel index (z n1 + y) n0 + x):
//   S      18 half spectra, [c][kz][ky][kx], kx < n0/2 (x-Nyquist dropped:
//          the Green operator zeroes it), complex T
//   E      current strain e (c = 0..8) and curvature gamma (c = 9..17), T
//   Eprev  the same fields one committed step earlier (extrapolation)
//   base   history base t_n - A e_n (0..8), m_n - B gamma_n (9..17), T
//   pq     p_n, q_n of the last committed step, FP64
//
// Per iteration: k_xpass<ITER> (x inverse, +E/Gamma, Alg. 1 twice for the
// error measure, polarization, x forward) -> k_axis (y fwd) -> k_axis
// (z fwd) -> k_green -> k_axis (z inv) -> k_axis (y inv) -> k_err_reduce.
// Every iteration kernel returns at once when the step's control block says
// the loop is finished, so batches of iterations can be queued ahead.
#pragma once

#include "device_math.hpp"

namespace mp {

constexpr int kMaxPts = 8;       // FFT points a thread holds in one stage
constexpr int kNPart = 30;       // per-block partials of the error measure (2 levels x 15)
constexpr int kNAvg = 40;        // per-block partials of the step averages

struct ErrMacro {
  double v[18];   // prescribed E then Gamma of the step
};

struct Ctl {
  int done;       // 0 running, 1 converged / fixed count reached, 2 max_iter, 3 diverged
  int iters;      // loop iterations of the current step
  int fixed;      // > 0: run exactly this many iterations
  int max_iter;
  double err;
  double tol;
  int norm;       // 0 local (Eq. 38), 1 average (Eq. 37)
  int pad;
  double err_parts[4];
};

enum XMode { X_ITER = 0, X_INIT = 1, X_FWD_ONLY = 2, X_INV_ONLY = 3 };

template <class T>
struct XArgs {
  int n0, n1, n2, nh, rows;
  uint32_t sched;
  const cx<T>* tw;
  cx<T>* S;
  long nspec, nvox;
  T* E;
  T* Eprev;
  const T* base;
  const double* pq;
  const uint8_t* phase;
  const PhaseC* params;
  double* partials;
  const Ctl* ctl;
  RefC ref;
  double mac[18];   // E then Gamma of the step
  double r;         // extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
  int first;        // first step of the plan: start from the uniform mac
  const T* fin;     // X_FWD_ONLY input (18 n)
  T* fout;          // X_INV_ONLY output (18 n)
};

// deterministic sum over a 64-lane wavefront (every lane gets the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// x pass: rows of n0 voxels, all 18 components.  LDS holds 9 packed complex
// pencils per row: pencil q = field 2q + i field 2q+1 (two real transforms
// in one complex transform).  Two lanes per voxel: lane level 0 runs the
// macro level of Alg. 1 (e -> t, tau), level 1 the micro level (gamma -> m,
// mu); the levels are independent, which halves each lane's live state.
// Each lane prefetches its old strain, history base and p_n / q_n before
// the transforms so the loads overlap them.
constexpr int kLev = 15;   // per-level partials: see k_xpass
template <class T, int MODE>
__global__ void __launch_bounds__(512) k_xpass(XArgs<T> a) {
  if (a.ctl && a.ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  T* ldr = reinterpret_cast<T*>(smem_raw);   // scalar view: field c of voxel v at 2 (q n0 ...) + (c & 1)
  __shared__ double red[8][2][kLev];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n0 = a.n0, nh = a.nh, rows = a.rows;
  const int vpb = rows * n0;
  const long row0 = (long)blockIdx.x * rows;
  const int npk = 9 * rows;
  // lanes [0, vpad) run the macro level, [vpad, 2 vpad) the micro level;
  // vpad is a multiple of 64, so the level is uniform over each wavefront
  const int vpad = nthr >> 1;
  const int lvl = __builtin_amdgcn_readfirstlane(tid >= vpad ? 1 : 0);
  const int v = tid - lvl * vpad;
  const bool own = v < vpb;
  const int vr = own ? v / n0 : 0, vx = own ? v % n0 : 0;
  // 32-bit voxel offset into wave-uniform component bases (the grid holds
  // at most 2^24 voxels)
  const int gi = int((row0 + vr) * n0 + vx);
  const long nv = a.nvox;
  T* const Elv = a.E + (long)lvl * 9 * nv;
  const T* const Blv = a.base + (long)lvl * 9 * nv;

  // prefetch this lane's history (ITER, INIT)
  T eo[9], bb[9];
  double hn = 0.0;
  int ph = 0;
  if ((MODE == X_ITER || MODE == X_INIT) && own) {
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      eo[c] = Elv[c * nv + gi];
      bb[c] = Blv[c * nv + gi];
    }
    hn = a.pq[lvl * nv + gi];
    ph = a.phase[gi];
  }

  if (MODE == X_ITER || MODE == X_INV_ONLY) {
    // half spectra -> packed full spectra Z = A + i B, Z(n0 - k) = conj A + i conj B
    for (int w = tid; w < npk * nh; w += nthr) {
      const int kx = w % nh, q = (w / nh) % 9, r = w / (nh * 9);
      const long off = (row0 + r) * nh + kx;
      const cx<T> A = a.S[(2 * q) * a.nspec + off];
      const cx<T> B = a.S[(2 * q + 1) * a.nspec + off];
      cx<T>* pen = lds + (r * 9 + q) * n0;
      pen[kx] = cx<T>{A.re - B.im, A.im + B.re};
      if (kx > 0)
        pen[n0 - kx] = cx<T>{A.re + B.im, B.re - A.im};
      else
        pen[nh] = cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_inplace<T, true, 8>(lds, n0, npk, 1, n0, false, a.sched, a.tw, tid, nthr);
  }

  // LDS scalar slot of field c (0..17) of this lane's voxel
  auto slot = [&](int c) { return 2 * ((vr * 9 + (c >> 1)) * n0 + vx) + (c & 1); };

  if (MODE == X_INV_ONLY) {
    if (own)
#pragma unroll
      for (int c = 0; c < 9; ++c) a.fout[(lvl * 9 + c) * nv + gi] = ldr[slot(lvl * 9 + c)];
    return;
  }

  // per-level partials of the error measure: |da|, |db| (max), |da|, |db| (sum),
  // |a|^2, |b|^2, b (sum), with (a, b) = (e, t) on the macro level and
  // (gamma, m) on the micro level.  Reduced over the wavefront as soon as
  // they exist (fixed butterfly order), then over the waves in order.
  const int lane = tid & 63, wv = tid >> 6, nw = (nthr + 63) >> 6;
  auto wave_put = [&](int j, double x) {
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      const double y = (lvl == L && own) ? x : 0.0;
      const double z = (j < 2) ? wave_max(y) : wave_sum(y);
      if (lane == 0) red[wv][L][j] = z;
    }
  };

  {
    T e[9];
    if (own) {
      if (MODE == X_FWD_ONLY) {
#pragma unroll
        for (int c = 0; c < 9; ++c) e[c] = a.fin[(lvl * 9 + c) * nv + gi];
      } else if (MODE == X_ITER) {
#pragma unroll
        for (int c = 0; c < 9; ++c) e[c] = ldr[slot(lvl * 9 + c)] + T(a.mac[lvl * 9 + c]);
      } else {  // X_INIT: first iterate of the step (Alg. 2)
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const long at = (lvl * 9 + c) * nv + gi;
          const T old = a.Eprev[at];
          e[c] = a.first ? T(a.mac[lvl * 9 + c]) : T(eo[c] + T(a.r) * (eo[c] - old));
          a.Eprev[at] = eo[c];
        }
      }
    }
    if (MODE == X_FWD_ONLY) {
      if (own)
#pragma unroll
        for (int c = 0; c < 9; ++c) ldr[slot(lvl * 9 + c)] = e[c];
    } else {
      // this lane's half of the phase record
      MacroC ct;
      MicroC cm;
      if (lvl == 0)
        ct = a.params[ph].t;
      else
        cm = a.params[ph].m;
      T t[9];
      double pnew;
      if (own) {
        if (lvl == 0)
          macro_return<T>(ct, e, bb, hn, t, pnew);
        else
          micro_return<T>(cm, e, bb, hn, t, pnew);
        // polarization (Eq. 34): tau = t - A0 e ; mu = m - B0 gamma
        T r0[9];
        if (lvl == 0)
          apply_A<T>(T(a.ref.lam), T(a.ref.mu), T(a.ref.kap), e, r0);
        else
          apply_B<T>(T(a.ref.alp), T(a.ref.bet), T(a.ref.gam), e, r0);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          ldr[slot(lvl * 9 + c)] = t[c] - r0[c];
          Elv[c * nv + gi] = e[c];
        }
      }
      if (MODE == X_ITER) {
        double da = 0, sa = 0, sb = 0;
        if (own)
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const double x = double(e[c]) - double(eo[c]);
            da += x * x;
            sa += double(e[c]) * double(e[c]);
            sb += double(t[c]) * double(t[c]);
          }
#pragma unroll
        for (int c = 0; c < 9; ++c) wave_put(6 + c, own ? double(t[c]) : 0.0);
        wave_put(4, sa);
        wave_put(5, sb);
        da = sqrt(da);
        wave_put(0, da);
        wave_put(2, da);
        // the old iterate's stresses, recomputed from the old strain (Alg. 1)
        double db = 0;
        if (own) {
          T to[9];
          double pold;
          if (lvl == 0)
            macro_return<T>(ct, eo, bb, hn, to, pold);
          else
            micro_return<T>(cm, eo, bb, hn, to, pold);
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const double y = double(t[c]) - double(to[c]);
            db += y * y;
          }
        }
        db = sqrt(db);
        wave_put(1, db);
        wave_put(3, db);
        __syncthreads();
        if (tid < 2 * kLev) {
          const int L = tid / kLev, j = tid % kLev;
          double y = red[0][L][j];
          for (int w = 1; w < nw; ++w) y = (j < 2) ? fmax(y, red[w][L][j]) : y + red[w][L][j];
          a.partials[(long)tid * gridDim.x + blockIdx.x] = y;
        }
      }
    }
  }
  __syncthreads();
  fft_inplace<T, false, 8>(lds, n0, npk, 1, n0, false, a.sched, a.tw, tid, nthr);
  // unpack: A = (Z(k) + conj Z(-k)) / 2, B = (Z(k) - conj Z(-k)) / (2 i)
  for (int w = tid; w < npk * nh; w += nthr) {
    const int kx = w % nh, q = (w / nh) % 9, r = w / (nh * 9);
    const cx<T>* pen = lds + (r * 9 + q) * n0;
    const cx<T> zk = pen[kx];
    const cx<T> zm = pen[kx == 0 ? 0 : n0 - kx];
    const long off = (row0 + r) * nh + kx;
    a.S[(2 * q) * a.nspec + off] = cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
    a.S[(2 * q + 1) * a.nspec + off] = cx<T>{T(0.5) * (zk.im + zm.im), T(0.5) * (zm.re - zk.re)};
  }

}

// error measure, stage 1: block j reduces partial row j over the x-pass blocks
__global__ void __launch_bounds__(256) k_err_rows(const double* partials, int nblk, double* tot,
                                                  const Ctl* ctl) {
  if (ctl->done) return;
  __shared__ double red[4];
  const int j = blockIdx.x, tid = threadIdx.x;
  const bool mx = (j % kLev) < 2;
  const double* row = partials + (long)j * nblk;
  double v0 = 0.0, v1 = 0.0;
  int b = tid;
  for (; b + 256 < nblk; b += 512) {
    const double x = row[b], y = row[b + 256];
    v0 = mx ? fmax(v0, x) : v0 + x;
    v1 = mx ? fmax(v1, y) : v1 + y;
  }
  if (b < nblk) v0 = mx ? fmax(v0, row[b]) : v0 + row[b];
  double v = mx ? fmax(v0, v1) : v0 + v1;
  v = mx ? wave_max(v) : wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0)
    tot[j] = mx ? fmax(fmax(red[0], red[1]), fmax(red[2], red[3]))
                : ((red[0] + red[1]) + (red[2] + red[3]));
}

// error measure, stage 2 (Eqs. 36-38).  <e> = E and <gamma> = Gamma hold
// exactly (the Green operator leaves no k = 0 fluctuation), so the averages
// of the strain-like fields are the prescribed ones.
__global__ void k_err_final(const double* tot, long nvox, Ctl* ctl, ErrMacro mac) {
  if (ctl->done || threadIdx.x != 0) return;
  const double inv = 1.0 / double(nvox);
  double err = 0.0;
  for (int f = 0; f < 4; ++f) {   // e, t, gamma, m
    const int L = f / 2, b = f % 2;
    const double* P = tot + L * kLev;
    const double num = ctl->norm == 0 ? P[b] : P[2 + b] * inv;
    double ea = 0.0;
    if (num != 0.0) {
      double mn = 0.0;
      for (int c = 0; c < 9; ++c) {
        const double mc = b == 0 ? mac.v[L * 9 + c] : P[6 + c] * inv;
        mn += mc * mc;
      }
      double den = sqrt(mn);
      const double rms = sqrt(P[4 + b] * inv);
      if (den <= 1e-6 * rms) den = rms;
      ea = num / den;
    }
    ctl->err_parts[f] = ea;
    err = (ea > err || ea != ea) ? ea : err;
  }
  ctl->err = err;
  const int it = ctl->iters + 1;
  ctl->iters = it;
  int done = 0;
  if (ctl->fixed > 0) {
    if (it >= ctl->fixed) done = 1;
  } else if (!(err <= 1e4)) {
    done = 3;
  } else if (err <= ctl->tol) {
    done = 1;
  } else if (it >= ctl->max_iter) {
    done = 2;
  }
  ctl->done = done;
}

// y or z pass over the half spectra: tile of L points x TX consecutive kx.
template <class T>
struct AxisArgs {
  cx<T>* S;
  long nspec;
  long ostride;    // stride of blockIdx.y
  long pstride;    // stride between points of the transformed axis
  int L, TX;
  uint32_t sched;
  const cx<T>* tw;
  const Ctl* ctl;
};

template <class T, bool INV>
__global__ void __launch_bounds__(256) k_axis(AxisArgs<T> a) {
  if (a.ctl && a.ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = a.L, TX = a.TX;
  cx<T>* g = a.S + (long)blockIdx.z * a.nspec + (long)blockIdx.y * a.ostride + (long)blockIdx.x * TX;
  for (int w = tid; w < L * TX; w += nthr) {
    const int i = w / TX, b = w % TX;
    lds[i * TX + b] = g[i * a.pstride + b];
  }
  __syncthreads();
  fft_inplace<T, INV, kMaxPts>(lds, L, TX, TX, 1, true, a.sched, a.tw, tid, nthr);
  for (int w = tid; w < L * TX; w += nthr) {
    const int i = w / TX, b = w % TX;
    g[i * a.pstride + b] = lds[i * TX + b];
  }
}

template <class T>
struct GreenArgs {
  cx<T>* S;
  long nspec;
  int n0, n1, n2, nh;
  double h, scale;
  RefC ref;
  const Ctl* ctl;
};

template <class T>
__global__ void __launch_bounds__(256) k_green(GreenArgs<T> a) {
  if (a.ctl && a.ctl->done) return;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.nspec) return;
  const int kx = int(idx % a.nh);
  const int ky = int((idx / a.nh) % a.n1);
  const int kz = int(idx / ((long)a.nh * a.n1));
  cx<T> tau[9], mu[9];
  const bool zero = (kx == 0 && ky == 0 && kz == 0) || (2 * ky == a.n1) || (2 * kz == a.n2);
  if (zero) {
#pragma unroll
    for (int c = 0; c < 18; ++c) a.S[c * a.nspec + idx] = cx<T>{T(0), T(0)};
    return;
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    tau[c] = a.S[c * a.nspec + idx];
    mu[c] = a.S[(9 + c) * a.nspec + idx];
  }
  const double tp = 6.283185307179586476925286766559;
  const int my = (2 * ky < a.n1) ? ky : ky - a.n1;
  const int mz = (2 * kz < a.n2) ? kz : kz - a.n2;
  const T x1 = T(tp * kx / (a.n0 * a.h));
  const T x2 = T(tp * my / (a.n1 * a.h));
  const T x3 = T(tp * mz / (a.n2 * a.h));
  green_apply<T>(a.ref, x1, x2, x3, T(a.scale), tau, mu);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    a.S[c * a.nspec + idx] = tau[c];
    a.S[(9 + c) * a.nspec + idx] = mu[c];
  }
}

__global__ void k_ctl_reset(Ctl* ctl, int fixed, int max_iter, double tol, int norm) {
  ctl->done = 0;
  ctl->iters = 0;
  ctl->fixed = fixed;
  ctl->max_iter = max_iter;
  ctl->err = 2.0 * tol;
  ctl->tol = tol;
  ctl->norm = norm;
}

// commit (last line of the step loop): final return map, new history base,
// output fields and the step averages.
template <class T>
struct CommitArgs {
  long nvox;
  const T* E;
  T* base;
  double* pq;
  T* out_tm;
  double* out_pq;
  const uint8_t* phase;
  const PhaseC* params;
  double* partials;
};

template <class T>
__global__ void __launch_bounds__(256) k_commit(CommitArgs<T> a) {
  __shared__ double red[4][kNAvg];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long gi = (long)blockIdx.x * blockDim.x + tid;
  double acc[kNAvg];
#pragma unroll
  for (int j = 0; j < kNAvg; ++j) acc[j] = 0.0;
  if (gi < a.nvox) {
    T e[18], bt[9], bm[9], t[9], m[9];
#pragma unroll
    for (int c = 0; c < 18; ++c) e[c] = a.E[c * a.nvox + gi];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      bt[c] = a.base[c * a.nvox + gi];
      bm[c] = a.base[(9 + c) * a.nvox + gi];
    }
    const PhaseC pc = a.params[a.phase[gi]];
    double p, q;
    return_map<T>(pc, e, e + 9, bt, bm, a.pq[gi], a.pq[a.nvox + gi], t, m, p, q);
    T ae[9], bg[9];
    apply_A<T>(T(pc.t.lam), T(pc.t.mu), T(pc.t.kap), e, ae);
    apply_B<T>(T(pc.m.alp), T(pc.m.bet), T(pc.m.gam), e + 9, bg);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      a.base[c * a.nvox + gi] = t[c] - ae[c];
      a.base[(9 + c) * a.nvox + gi] = m[c] - bg[c];
      a.out_tm[c * a.nvox + gi] = t[c];
      a.out_tm[(9 + c) * a.nvox + gi] = m[c];
      acc[c] = double(t[c]);
      acc[9 + c] = double(m[c]);
      acc[18 + c] = double(e[c]);
      acc[27 + c] = double(e[9 + c]);
    }
    a.pq[gi] = p;
    a.pq[a.nvox + gi] = q;
    a.out_pq[gi] = p;
    a.out_pq[a.nvox + gi] = q;
    double teq, meq;
    equivalent_stresses<T>(pc, t, m, teq, meq);
    acc[36] = p;
    acc[37] = q;
    acc[38] = teq;
    acc[39] = meq;
  }
#pragma unroll
  for (int j = 0; j < kNAvg; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[wv][j] = v;
  }
  __syncthreads();
  if (tid < kNAvg) {
    const double v = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    a.partials[(long)blockIdx.x * kNAvg + tid] = v;
  }
}

__global__ void __launch_bounds__(256) k_avg_reduce(const double* partials, int nblk, long nvox,
                                                    double* resp) {
  __shared__ double red[4][kNAvg];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = 0; j < kNAvg; ++j) {
    double v = 0.0;
    for (int b = tid; b < nblk; b += 256) v += partials[(long)b * kNAvg + j];
    v = wave_sum(v);
    if (lane == 0) red[wv][j] = v;
  }
  __syncthreads();
  if (tid < kNAvg) {
    const double v = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    resp[tid] = v / double(nvox);
  }
}

// pointwise Alg. 1 on independent points (same device code as the solver)
template <class T>
__global__ void __launch_bounds__(256) k_rrm_points(long n, const uint8_t* phase, const PhaseC* params,
                                                    const T* e, const T* g, const T* en, const T* gn,
                                                    const T* tn, const T* mn, const double* pn,
                                                    const double* qn, T* t, T* m, double* p, double* q) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PhaseC pc = params[phase[i]];
  T ev[18], env[18], bt[9], bm[9], ae[9], bg[9], to[9], mo[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    ev[c] = e[c * n + i];
    ev[9 + c] = g[c * n + i];
    env[c] = en[c * n + i];
    env[9 + c] = gn[c * n + i];
  }
  apply_A<T>(T(pc.t.lam), T(pc.t.mu), T(pc.t.kap), env, ae);
  apply_B<T>(T(pc.m.alp), T(pc.m.bet), T(pc.m.gam), env + 9, bg);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    bt[c] = tn[c * n + i] - ae[c];
    bm[c] = mn[c * n + i] - bg[c];
  }
  double pp, qq;
  return_map<T>(pc, ev, ev + 9, bt, bm, pn[i], qn[i], to, mo, pp, qq);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    t[c * n + i] = to[c];
    m[c * n + i] = mo[c];
  }
  p[i] = pp;
  q[i] = qq;
}

}  // namespace mp
