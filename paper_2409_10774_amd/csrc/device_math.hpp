// Device building blocks of the micropolar FFT solver (gfx950).
//
//   cx<T>            interleaved complex value (re, im), 2*sizeof(T) aligned
//   fft_ct           self-sorting mixed-radix Stockham FFT of a batch of
//                    pencils held in LDS (radices 8, 4, 2, 3), all sizes
//                    compile-time; each stage gathers its butterflies into
//                    registers, barriers, then scatters, so one LDS buffer
//                    suffices
//   PhaseC           per-phase constants with the derived a2, b2 of Alg. 1
//   return_map       micropolar radial return of Alg. 1 at one voxel
//   green_apply      reference-medium Green operator at one frequency
//                    (closed-form solve of the 6x6 Fourier symbol of the
//                    balance equations, Eqs. 1, 2, 6, 33-35)
//   green_apply_gen  the same for a general (Eq. 5) reference medium: the
//                    symbol assembled from stored coefficients and factored
//   green_symbol_inverse, green_apply_stored
//                    the Green operator stored per frequency (Sec. 2.4):
//                    the inverse symbol's 21 entries, computed once, then
//                    applied from the table
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

template <class T>
struct __align__(2 * sizeof(T)) cx {
  T re, im;
};

// Global-memory pointers.  A pointer read out of device memory (a batch
// descriptor) carries no address space, and accesses through it compile to
// flat instructions, which also hold the LDS wait counter.  Every global
// access of the passes goes through a pointer typed for the global address
// space instead.
#define MP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MP_GLOBAL T* glob(T* p) {
  return (MP_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const MP_GLOBAL T* glob(const T* p) {
  return (const MP_GLOBAL T*)p;
}
// Read-only memory through the constant address space: loads at a
// wave-uniform address become scalar loads.
#define MP_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const MP_CONST T* cnst(const T* p) {
  return (const MP_CONST T*)p;
}

// complex values and constant records move through global memory as whole
// vector words (one dwordx2 / dwordx4 access per complex value)
template <class T>
struct Vec2;
template <>
struct Vec2<float> {
  typedef float __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec2<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};
template <class T>
__device__ __forceinline__ cx<T> gload(const MP_GLOBAL cx<T>* p) {
  const typename Vec2<T>::type v = *(const MP_GLOBAL typename Vec2<T>::type*)p;
  return cx<T>{v.x, v.y};
}
template <class T>
__device__ __forceinline__ void gstore(MP_GLOBAL cx<T>* p, cx<T> v) {
  typename Vec2<T>::type w;
  w.x = v.re;
  w.y = v.im;
  *(MP_GLOBAL typename Vec2<T>::type*)p = w;
}
// copy an N-entry twiddle table from global memory into LDS (visible after
// the caller's next barrier)
template <class T, int N, int NTHR>
__device__ __forceinline__ void load_twiddles(cx<T>* twl, const MP_GLOBAL cx<T>* tw, int tid) {
  for (int i = tid; i < N; i += NTHR) twl[i] = gload(tw + i);
}

template <class S>
__device__ __forceinline__ S gread(const MP_GLOBAL S* p) {
  static_assert(sizeof(S) % 8 == 0, "record of 8-byte words");
  S out;
  const MP_GLOBAL unsigned long long* q = (const MP_GLOBAL unsigned long long*)p;
  unsigned long long* o = reinterpret_cast<unsigned long long*>(&out);
#pragma unroll
  for (int i = 0; i < int(sizeof(S) / 8); ++i) o[i] = q[i];
  return out;
}

template <class T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward) or +i (inverse)
template <class T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}
template <class T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.im, a.re}; }

// ---------------------------------------------------------------------------
// small DFTs in registers: X_s = sum_r a_r exp(-+ 2 pi i r s / R)
// ---------------------------------------------------------------------------
template <class T, int R, bool INV>
struct Dft;

template <class T, bool INV>
struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <class T, bool INV>
struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    cx<T> t2 = cadd(a[1], a[3]), t3 = rot90<T, INV>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <class T, bool INV>
struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> ev[4] = {a[0], a[2], a[4], a[6]};
    cx<T> od[4] = {a[1], a[3], a[5], a[7]};
    Dft<T, 4, INV>::run(ev);
    Dft<T, 4, INV>::run(od);
    const T c = T(0.70710678118654752440084436210484903928);
    // W8^s with W8 = exp(-+ i pi / 4)
    cx<T> w1 = INV ? cx<T>{c, c} : cx<T>{c, -c};
    cx<T> w3 = INV ? cx<T>{-c, c} : cx<T>{-c, -c};
    cx<T> o0 = od[0];
    cx<T> o1 = cmul(od[1], w1);
    cx<T> o2 = rot90<T, INV>(od[2]);
    cx<T> o3 = cmul(od[3], w3);
    a[0] = cadd(ev[0], o0);
    a[4] = csub(ev[0], o0);
    a[1] = cadd(ev[1], o1);
    a[5] = csub(ev[1], o1);
    a[2] = cadd(ev[2], o2);
    a[6] = csub(ev[2], o2);
    a[3] = cadd(ev[3], o3);
    a[7] = csub(ev[3], o3);
  }
};

template <class T, bool INV>
struct Dft<T, 3, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    const T h = T(0.86602540378443864676372317075293618347);  // sqrt(3) / 2
    cx<T> s = cadd(a[1], a[2]);
    cx<T> d = csub(a[1], a[2]);
    cx<T> m = {a[0].re - T(0.5) * s.re, a[0].im - T(0.5) * s.im};
    cx<T> r = rot90<T, INV>(cx<T>{d.re * h, d.im * h});
    a[0] = cadd(a[0], s);
    a[1] = cadd(m, r);
    a[2] = csub(m, r);
  }
};

// ---------------------------------------------------------------------------
// Self-sorting mixed-radix Stockham FFT, in place in LDS, every size and
// stride a compile-time constant (index arithmetic folds to shifts and
// multiplies).
//   pencil b, point i lives at buf[b * BS + i * PS]; N points per pencil,
//   NB pencils, NTHR threads.  P = product of the radices already applied.
//   Butterfly w reads points i + r N/R, twiddles them by
//   exp(-+2 pi i r k / (P R)), k = i mod P, runs an R-point DFT and writes
//   points (i - k) R + k + s P.  Every thread gathers all its butterflies
//   into registers, the block barriers, then scatters, so one buffer is
//   enough.  Radices: 8 while it divides, then 4, 2, 3.
//   tw: N-entry table exp(-2 pi i m / N), held in LDS.  Unnormalised in both
//   directions.
// ---------------------------------------------------------------------------
template <class T, int R, bool INV, int N, int P, int NB, int PS, int BS, bool BFAST, int NTHR>
__device__ __forceinline__ void stage_ct(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  constexpr int NBF = N / R;
  constexpr int TOTAL = NBF * NB;
  constexpr int MB = (TOTAL + NTHR - 1) / NTHR;
  constexpr int TWS = N / (P * R);
  cx<T> u[MB][R];
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    const int w = tid + j * NTHR;
    if (TOTAL % NTHR == 0 || w < TOTAL) {
      const int b = BFAST ? w % NB : w / NBF;
      const int i = BFAST ? w / NB : w % NBF;
      const cx<T>* src = buf + b * BS + i * PS;
#pragma unroll
      for (int r = 0; r < R; ++r) u[j][r] = src[r * NBF * PS];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    const int w = tid + j * NTHR;
    if (TOTAL % NTHR == 0 || w < TOTAL) {
      const int b = BFAST ? w % NB : w / NBF;
      const int i = BFAST ? w / NB : w % NBF;
      const int k = i % P;
      if (P > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> t = tw[r * k * TWS];
          if (INV) t.im = -t.im;
          u[j][r] = cmul(u[j][r], t);
        }
      }
      Dft<T, R, INV>::run(u[j]);
      cx<T>* dst = buf + b * BS + ((i - k) * R + k) * PS;
#pragma unroll
      for (int s = 0; s < R; ++s) dst[s * P * PS] = u[j][s];
    }
  }
  __syncthreads();
}

template <int REM>
struct NextRadix {
  static constexpr int value = REM % 8 == 0 ? 8 : REM % 4 == 0 ? 4 : REM % 2 == 0 ? 2 : 3;
};

template <class T, bool INV, int N, int P, int NB, int PS, int BS, bool BFAST, int NTHR>
__device__ __forceinline__ void fft_ct(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  if constexpr (P < N) {
    constexpr int R = NextRadix<N / P>::value;
    static_assert((N / P) % R == 0, "size must be a product of 2s and 3s");
    stage_ct<T, R, INV, N, P, NB, PS, BS, BFAST, NTHR>(buf, tw, tid);
    fft_ct<T, INV, N, P * R, NB, PS, BS, BFAST, NTHR>(buf, tw, tid);
  }
}

// Out-of-place variant (ping-pong between two LDS buffers): each stage reads
// src and writes dst, so one barrier per stage suffices (the in-place stage
// needs two).  fft_pp_stages<N>() stages; the result ends in `a` when that
// count is even, else in `b`.  Entry: the data in `a`, visible to the block.
template <int N, int P = 1>
constexpr int fft_pp_stages() {
  if constexpr (P >= N) {
    return 0;
  } else {
    return 1 + fft_pp_stages<N, P * NextRadix<N / P>::value>();
  }
}

template <class T, int R, bool INV, int N, int P, int NB, int PS, int BS, bool BFAST, int NTHR>
__device__ __forceinline__ void stage_pp(const cx<T>* src, cx<T>* dst, const cx<T>* __restrict__ tw,
                                         int tid) {
  constexpr int NBF = N / R;
  constexpr int TOTAL = NBF * NB;
  constexpr int MB = (TOTAL + NTHR - 1) / NTHR;
  constexpr int TWS = N / (P * R);
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    const int w = tid + j * NTHR;
    if (TOTAL % NTHR == 0 || w < TOTAL) {
      const int b = BFAST ? w % NB : w / NBF;
      const int i = BFAST ? w / NB : w % NBF;
      const int k = i % P;
      cx<T> u[R];
      const cx<T>* s = src + b * BS + i * PS;
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = s[r * NBF * PS];
      if (P > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> t = tw[r * k * TWS];
          if (INV) t.im = -t.im;
          u[r] = cmul(u[r], t);
        }
      }
      Dft<T, R, INV>::run(u);
      cx<T>* d = dst + b * BS + ((i - k) * R + k) * PS;
#pragma unroll
      for (int r = 0; r < R; ++r) d[r * P * PS] = u[r];
    }
  }
  __syncthreads();
}

template <class T, bool INV, int N, int P, int NB, int PS, int BS, bool BFAST, int NTHR>
__device__ __forceinline__ void fft_pp(cx<T>* a, cx<T>* b, const cx<T>* __restrict__ tw, int tid) {
  if constexpr (P < N) {
    constexpr int R = NextRadix<N / P>::value;
    static_assert((N / P) % R == 0, "size must be a product of 2s and 3s");
    stage_pp<T, R, INV, N, P, NB, PS, BS, BFAST, NTHR>(a, b, tw, tid);
    fft_pp<T, INV, N, P * R, NB, PS, BS, BFAST, NTHR>(b, a, tw, tid);
  }
}

// ---------------------------------------------------------------------------
// Alg. 1: micropolar radial return at one voxel.
// ---------------------------------------------------------------------------
// Constants of one phase, split by level so a lane loads only its half.
struct MacroC {
  double lam, mu, kap;   // Eq. 6 moduli of A
  double tY, tH;         // Eq. 15 yield stress and hardening
  double a1, a2;         // Eq. 14 weights, a2 = a1 mu / kappa (Alg. 1)
  double aid;            // index of the phase's Eq. 5 tensors, -1 for Eq. 6
};
struct MicroC {
  double alp, bet, gam;  // Eq. 6 moduli of B
  double mY, mH;         // Eq. 18 yield stress and hardening
  double b1;             // Eq. 17 weight
  double b2;             // b1 (gamma + beta) / (gamma - beta); 0 when gamma == beta
  double b2gmb;          // b2 (gamma - beta); b1 (gamma + beta) when gamma == beta
};
struct PhaseC {
  MacroC t;
  MicroC m;
};

// Eq. 5 with general tensors: out_i = R_ij x_j for a 9 x 9 row matrix R
// (FP64 in global memory), i = 3k + l, j = 3m + n
// Row-matrix product out = R x of an Eq. 5 law (R in the constant address
// space: a wave-uniform R is read through the scalar cache).
template <class T>
__device__ __forceinline__ void aniso_apply(const MP_CONST double* R, const T* x, T* out) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    T s = T(0);
#pragma unroll
    for (int j = 0; j < 9; ++j) s += T(R[9 * i + j]) * x[j];
    out[i] = s;
  }
}

// The Eq. 5 law of this lane's record aid (0 <= aid < n) at level lvl
// (wave-uniform) of the table [record][level][81].  The records are visited
// in a wave-uniform loop so that each one's rows are read at a wave-uniform
// address; the match is made opaque, or the compiler would address the rows
// by the equal per-lane aid.
template <class T>
__device__ __forceinline__ void aniso_apply_wave(const double* table, int n, int aid, int lvl, const T* x,
                                                 T* out) {
  for (int j = 0; j < n; ++j) {
    int hit = aid == j;
    asm volatile("" : "+v"(hit));
    if (hit) aniso_apply<T>(cnst(table) + (2L * j + lvl) * 81, x, out);
  }
}

// t_kl = lam tr(e) d_kl + (mu + kappa) e_kl + (mu - kappa) e_lk      (Eq. 6)
template <class T>
__device__ __forceinline__ void apply_A(T lam, T mu, T kap, const T* e, T* t) {
  const T tr = e[0] + e[4] + e[8];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      t[3 * k + l] = (mu + kap) * e[3 * k + l] + (mu - kap) * e[3 * l + k] + (k == l ? lam * tr : T(0));
}

// m_kl = B_lkmn g_mn = alpha tr(g) d_kl + beta g_kl + gamma g_lk       (Eq. 6)
template <class T>
__device__ __forceinline__ void apply_B(T alp, T bet, T gam, const T* g, T* m) {
  const T tr = g[0] + g[4] + g[8];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      m[3 * k + l] = bet * g[3 * k + l] + gam * g[3 * l + k] + (k == l ? alp * tr : T(0));
}

// Macro level of Alg. 1 at one voxel: trial stress from the history base
// bt = t_n - A e_n (Eq. 30: t_trial = t_n + A (e - e_n) = bt + A e), Eq. 14
// equivalent stress, closed-form p of Eq. 32, radial scaling of the
// deviatoric sym / skew parts.
template <class T>
__device__ __forceinline__ void macro_return(const MacroC& c, const T* e, const T* bt, double pn,
                                             T* t, double& p) {
  apply_A<T>(T(c.lam), T(c.mu), T(c.kap), e, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) t[i] += bt[i];
  const T vol = (t[0] + t[4] + t[8]) / T(3);
  T ss[9], sk[9];
  T n_sym = 0, n_skw = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const T skl = t[3 * k + l] - (k == l ? vol : T(0));
      const T slk = t[3 * l + k] - (k == l ? vol : T(0));
      ss[3 * k + l] = T(0.5) * (skl + slk);
      sk[3 * k + l] = T(0.5) * (skl - slk);
      n_sym += ss[3 * k + l] * ss[3 * k + l];
      n_skw += sk[3 * k + l] * sk[3 * k + l];
    }
  const double teq = sqrt(c.a1 * double(n_sym) + c.a2 * double(n_skw));
  if (teq < c.tY + c.tH * pn) {
    p = pn;
  } else {
    const double den = c.tH + 2.0 * c.a1 * c.mu;
    p = pn * (2.0 * c.a1 * c.mu) / den + (teq - c.tY) / den;
    const double R1 = c.tY + c.tH * p;
    const T fs = T(R1 / (R1 + 2.0 * (p - pn) * c.a1 * c.mu));
    const T fk = T(R1 / (R1 + 2.0 * (p - pn) * c.a2 * c.kap));
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l)
        t[3 * k + l] = (k == l ? vol : T(0)) + fs * ss[3 * k + l] + fk * sk[3 * k + l];
  }
}

// Micro level of Alg. 1: trial couple stress bm + B g, Eq. 17 on the full
// couple stress, closed-form q of Eq. 32, radial scaling of sym / skew parts.
template <class T>
__device__ __forceinline__ void micro_return(const MicroC& c, const T* g, const T* bm, double qn,
                                             T* m, double& q) {
  apply_B<T>(T(c.alp), T(c.bet), T(c.gam), g, m);
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] += bm[i];
  T ms[9], mk[9];
  T m_sym = 0, m_skw = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      ms[3 * k + l] = T(0.5) * (m[3 * k + l] + m[3 * l + k]);
      mk[3 * k + l] = T(0.5) * (m[3 * k + l] - m[3 * l + k]);
      m_sym += ms[3 * k + l] * ms[3 * k + l];
      m_skw += mk[3 * k + l] * mk[3 * k + l];
    }
  const double meq = sqrt(c.b1 * double(m_sym) + c.b2 * double(m_skw));
  if (meq < c.mY + c.mH * qn) {
    q = qn;
  } else {
    const double bgb = c.b1 * (c.gam + c.bet);
    const double den = c.mH + bgb;
    q = qn * bgb / den + (meq - c.mY) / den;
    const double R2 = c.mY + c.mH * q;
    const T gs = T(R2 / (R2 + (q - qn) * bgb));
    const T gk = T(R2 / (R2 + (q - qn) * c.b2gmb));
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = gs * ms[i] + gk * mk[i];
  }
}

// Alg. 1 at one voxel: the two levels are independent.
template <class T>
__device__ __forceinline__ void return_map(const PhaseC& c, const T* e, const T* g, const T* bt,
                                           const T* bm, double pn, double qn, T* t, T* m,
                                           double& p, double& q) {
  macro_return<T>(c.t, e, bt, pn, t, p);
  micro_return<T>(c.m, g, bm, qn, m, q);
}

// t_eq of a final state (Eq. 14), FP64
template <class T>
__device__ __forceinline__ double macro_equivalent(const MacroC& c, const T* t) {
  const double vol = (double(t[0]) + double(t[4]) + double(t[8])) / 3.0;
  double n_sym = 0, n_skw = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double skl = double(t[3 * k + l]) - (k == l ? vol : 0.0);
      const double slk = double(t[3 * l + k]) - (k == l ? vol : 0.0);
      n_sym += 0.25 * (skl + slk) * (skl + slk);
      n_skw += 0.25 * (skl - slk) * (skl - slk);
    }
  return sqrt(c.a1 * n_sym + c.a2 * n_skw);
}

// m_eq of a final state (Eq. 17), FP64
template <class T>
__device__ __forceinline__ double micro_equivalent(const MicroC& c, const T* m) {
  double m_sym = 0, m_skw = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double a = 0.5 * (double(m[3 * k + l]) + double(m[3 * l + k]));
      const double b = 0.5 * (double(m[3 * k + l]) - double(m[3 * l + k]));
      m_sym += a * a;
      m_skw += b * b;
    }
  return sqrt(c.b1 * m_sym + c.b2 * m_skw);
}

// Eq. 6 constants of an isotropic reference medium (the Green operator's
// A0, B0; the augmented-Lagrangian scheme's penalty)
struct RefC {
  double lam, mu, kap, alp, bet, gam;
};

// ---------------------------------------------------------------------------
// Local step of the augmented-Lagrangian scheme (the high-contrast scheme of
// Michel, Moulinec and Suquet that the paper's conclusion names), at one voxel
// and level: the strain d with  s(d) + C0 d = r,  s(d) the stress Alg. 1
// returns for d from the history base b, C0 the penalty (the reference
// medium).  Alg. 1 scales the deviator of the trial stress (macro level) or
// the whole trial couple stress (micro level) by one factor f, and with the
// isotropic laws of Eq. 6 the equation splits into the volumetric part
// tr(V) I / 3, the symmetric deviator and the skew part of each tensor, on
// which the law and the penalty act as scalars a_j, a0_j.  For a given f
//   d_j = (r_j - f b_j) / (f a_j + a0_j),  trial part T_j = u_j / (f a_j + a0_j),
//   u_j = a0_j b_j + a_j r_j,
// and f is the root in (0, 1] of the consistency condition of Alg. 1,
//   F(f) = (f - c1) X(f) - c0,  X = equivalent trial stress (Eq. 14 / 17),
//   c1 = H / (H + c),  c0 = R_n c / (H + c),
// which is increasing in f: safeguarded Newton steps inside a bracket.
// ---------------------------------------------------------------------------
// parts of a 3 x 3 tensor: volumetric scalar v (V = v I + D + K), symmetric
// deviator D, skew part K
__device__ __forceinline__ void tensor_parts(const double* V, double& v, double* D, double* K) {
  v = (V[0] + V[4] + V[8]) / 3.0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      D[3 * k + l] = 0.5 * (V[3 * k + l] + V[3 * l + k]) - (k == l ? v : 0.0);
      K[3 * k + l] = 0.5 * (V[3 * k + l] - V[3 * l + k]);
    }
}

__device__ __forceinline__ double norm2_9(const double* V) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) s += V[i] * V[i];
  return s;
}

// root in (0, 1] of F(f) = (f - c1) sqrt(w0 Q0 / (f p0 + q0)^2 + w1 Q1 /
// (f p1 + q1)^2 + w2 Q2 / (f p2 + q2)^2 + W) - c0 (F increasing, F(1) >= 0):
// Newton steps kept inside the bracket, bisection where a step leaves it.
// The first iterate is c1 + c0 / X1, X1 = X(1) the elastic trial value: the
// root with X frozen there, an upper bracket since X decreases in f.
__device__ __forceinline__ double al_factor(const double (&w)[3], const double (&Q)[3], const double (&p)[3],
                                            const double (&q)[3], double W, double c0, double c1, double X1) {
  double lo = 0.0, hi = 1.0, f = c1 + c0 / X1;
  if (!(f > 0.0 && f <= 1.0)) f = 1.0;
  for (int it = 0; it < 100; ++it) {
    double X2 = W, dX2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double id = 1.0 / (f * p[j] + q[j]);
      const double t = w[j] * Q[j] * id * id;
      X2 += t;
      dX2 -= 2.0 * t * p[j] * id;
    }
    const double X = sqrt(X2);
    const double F = (f - c1) * X - c0;
    if (F > 0.0) hi = f; else lo = f;
    if (F == 0.0) break;
    const double dF = X + (f - c1) * 0.5 * dX2 / X;
    double nf = f - F / dF;
    if (!(nf > lo && nf < hi)) nf = 0.5 * (lo + hi);
    if (fabs(nf - f) <= 1e-16 * f || hi - lo <= 1e-16 * hi) {
      f = nf;
      break;
    }
    f = nf;
  }
  return f;
}

// macro level: strain d of  t(d) + A0 d = r  (history base bt, p_n)
__device__ __forceinline__ void al_macro_local(const MacroC& c, const RefC& r0, const double* r,
                                               const double* bt, double pn, double* d) {
  const double a[3] = {3.0 * c.lam + 2.0 * c.mu, 2.0 * c.mu, 2.0 * c.kap};
  const double a0[3] = {3.0 * r0.lam + 2.0 * r0.mu, 2.0 * r0.mu, 2.0 * r0.kap};
  double rv, rD[9], rK[9], bv, bD[9], bK[9];
  tensor_parts(r, rv, rD, rK);
  tensor_parts(bt, bv, bD, bK);
  // the volumetric part is never scaled
  const double dv = (rv - bv) / (a[0] + a0[0]);
  double uD[9], uK[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    uD[i] = a0[1] * bD[i] + a[1] * rD[i];
    uK[i] = a0[2] * bK[i] + a[2] * rK[i];
  }
  const double QD = norm2_9(uD), QK = norm2_9(uK);
  // elastic trial (f = 1): Eq. 14 on the deviator
  const double sD = a[1] + a0[1], sK = a[2] + a0[2];
  const double X1 = sqrt(c.a1 * QD / (sD * sD) + c.a2 * QK / (sK * sK));
  const double Rn = c.tY + c.tH * pn;
  double f = 1.0;
  if (!(X1 < Rn)) {
    const double den = c.tH + 2.0 * c.a1 * c.mu;
    const double w[3] = {c.a1, c.a2, 0.0}, Q[3] = {QD, QK, 0.0};
    const double p[3] = {a[1], a[2], 0.0}, q[3] = {a0[1], a0[2], 1.0};
    f = al_factor(w, Q, p, q, 0.0, Rn * 2.0 * c.a1 * c.mu / den, c.tH / den, X1);
  }
  const double ieD = 1.0 / (f * a[1] + a0[1]), ieK = 1.0 / (f * a[2] + a0[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int i = 3 * k + l;
      d[i] = (rD[i] - f * bD[i]) * ieD + (rK[i] - f * bK[i]) * ieK + (k == l ? dv : 0.0);
    }
}

// micro level: curvature d of  m(d) + B0 d = r  (history base bm, q_n); a part
// without stiffness in the phase and the penalty (the skew curvature when
// gamma = beta and gamma0 = beta0) takes the compatible field's part, comp
__device__ __forceinline__ void al_micro_local(const MicroC& c, const RefC& r0, const double* r,
                                               const double* bm, const double* comp, double qn, double* d) {
  const double a[3] = {3.0 * c.alp + c.bet + c.gam, c.bet + c.gam, c.bet - c.gam};
  const double a0[3] = {3.0 * r0.alp + r0.bet + r0.gam, r0.bet + r0.gam, r0.bet - r0.gam};
  const bool inert = a[2] == 0.0 && a0[2] == 0.0;
  double rv, rD[9], rK[9], bv, bD[9], bK[9];
  tensor_parts(r, rv, rD, rK);
  tensor_parts(bm, bv, bD, bK);
  double uD[9], uK[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    uD[i] = a0[1] * bD[i] + a[1] * rD[i];
    uK[i] = a0[2] * bK[i] + a[2] * rK[i];
  }
  const double uv = a0[0] * bv + a[0] * rv;
  // Eq. 17 on the whole couple stress: b1 (|vol|^2 + |D|^2) + b2 |K|^2, the
  // volumetric part contributing 3 v^2
  const double Qv = 3.0 * uv * uv, QD = norm2_9(uD), QK = norm2_9(uK);
  const double W = inert ? c.b2 * norm2_9(bK) : 0.0;   // inert part: constant trial stress b
  const double s0 = a[0] + a0[0], s1 = a[1] + a0[1], s2 = a[2] + a0[2];
  const double Y1 = sqrt(c.b1 * Qv / (s0 * s0) + c.b1 * QD / (s1 * s1) + (inert ? W : c.b2 * QK / (s2 * s2)));
  const double Rn = c.mY + c.mH * qn;
  double g = 1.0;
  if (!(Y1 < Rn)) {
    const double bgb = c.b1 * (c.gam + c.bet);
    const double den = c.mH + bgb;
    const double w[3] = {c.b1, c.b1, inert ? 0.0 : c.b2};
    const double Q[3] = {Qv, QD, inert ? 0.0 : QK};
    const double p[3] = {a[0], a[1], inert ? 0.0 : a[2]}, q[3] = {a0[0], a0[1], inert ? 1.0 : a0[2]};
    g = al_factor(w, Q, p, q, W, Rn * bgb / den, c.mH / den, Y1);
  }
  const double ieD = 1.0 / (g * a[1] + a0[1]), ieK = inert ? 0.0 : 1.0 / (g * a[2] + a0[2]);
  double cv = 0.0, cD[9], cK[9];
  if (inert) tensor_parts(comp, cv, cD, cK);
  const double dv = (rv - g * bv) / (g * a[0] + a0[0]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int i = 3 * k + l;
      const double dk = inert ? cK[i] : (rK[i] - g * bK[i]) * ieK;
      d[i] = (rD[i] - g * bD[i]) * ieD + dk + (k == l ? dv : 0.0);
    }
}

// ---------------------------------------------------------------------------
// Green operator at one frequency.
//   Sources of the reference-medium balance equations (Eq. 2 with the
//   polarization as eigenstress): bu_l = i xi_k tau_kl,
//   bp_l = i xi_k mu_kl + eps_lkm tau_km.  The amplitudes (u, phi) of the
//   fluctuation solve K (u, phi) = (bu, bp) with K the 6x6 Hermitian Fourier
//   symbol of the reference medium; then e_kl = i xi_k u_l + eps_lkm phi_m and
//   g_kl = i xi_l phi_k (Eq. 1), scaled by `scale` (the inverse-DFT 1/N).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void green_sources(const T (&xi)[3], const cx<T>* tau, const cx<T>* mu,
                                              cx<T> (&bu)[3], cx<T> (&bp)[3]) {
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    cx<T> su = {0, 0}, sp = {0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      su = cadd(su, cscale(tau[3 * k + l], xi[k]));
      sp = cadd(sp, cscale(mu[3 * k + l], xi[k]));
    }
    bu[l] = mul_i(su);
    bp[l] = mul_i(sp);
  }
  // eps_lkm tau_km
  bp[0] = cadd(bp[0], csub(tau[5], tau[7]));
  bp[1] = cadd(bp[1], csub(tau[6], tau[2]));
  bp[2] = cadd(bp[2], csub(tau[1], tau[3]));
}

template <class T>
__device__ __forceinline__ void green_strains(const T (&xi)[3], const cx<T> (&u)[3], const cx<T> (&ph)[3],
                                              T scale, cx<T>* tau /*e out*/, cx<T>* mu /*g out*/) {
  // e_kl = i xi_k u_l + eps_lkm phi_m ; g_kl = i xi_l phi_k
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      tau[3 * k + l] = mul_i(cscale(u[l], xi[k]));
      mu[3 * k + l] = mul_i(cscale(ph[k], xi[l]));
    }
  tau[1] = csub(tau[1], ph[2]);
  tau[2] = cadd(tau[2], ph[1]);
  tau[3] = cadd(tau[3], ph[2]);
  tau[5] = csub(tau[5], ph[0]);
  tau[6] = csub(tau[6], ph[1]);
  tau[7] = cadd(tau[7], ph[0]);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    tau[i] = cscale(tau[i], scale);
    mu[i] = cscale(mu[i], scale);
  }
}

// Isotropic reference medium (Eq. 6 constants): the symbol is
//   K = [[(mu0+k0) s^2 I + (lam0+mu0-k0) xi xi^T, -2 i k0 W],
//        [-2 i k0 W, (g0 s^2 + 4 k0) I + (a0 + b0) xi xi^T]],  W v = xi x v,
// which splits into a longitudinal part along n = xi/s and a 2x2 transverse
// block, solved in closed form.

template <class T>
__device__ __forceinline__ void green_apply(const RefC& r, T x1, T x2, T x3, T scale,
                                            cx<T>* tau /*9 in, e out*/, cx<T>* mu /*9 in, g out*/) {
  const T xi[3] = {x1, x2, x3};
  cx<T> bu[3], bp[3];
  green_sources<T>(xi, tau, mu, bu, bp);

  const T s2 = x1 * x1 + x2 * x2 + x3 * x3;
  const T s = sqrt(s2);
  const T n[3] = {x1 / s, x2 / s, x3 / s};
  const T lam = T(r.lam), mu0 = T(r.mu), kap = T(r.kap), alp = T(r.alp), bet = T(r.bet),
          gam = T(r.gam);
  cx<T> nbu = {0, 0}, nbp = {0, 0};
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    nbu = cadd(nbu, cscale(bu[l], n[l]));
    nbp = cadd(nbp, cscale(bp[l], n[l]));
  }
  const T a = (mu0 + kap) * s2;
  const T c = gam * s2 + T(4) * kap;
  const T D = s2 * ((mu0 + kap) * gam * s2 + T(4) * mu0 * kap);
  const T iD = T(1) / D;
  const T iL = T(1) / ((lam + T(2) * mu0) * s2);
  const T iP = T(1) / ((alp + bet + gam) * s2 + T(4) * kap);
  const T ks2 = T(2) * kap * s;
  // n x b (the longitudinal part drops out of the cross product)
  cx<T> nxu[3], nxp[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int a1 = (l + 1) % 3, a2 = (l + 2) % 3;
    nxu[l] = csub(cscale(bu[a2], n[a1]), cscale(bu[a1], n[a2]));
    nxp[l] = csub(cscale(bp[a2], n[a1]), cscale(bp[a1], n[a2]));
  }
  cx<T> u[3], ph[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const cx<T> buT = csub(bu[l], cscale(nbu, n[l]));
    const cx<T> bpT = csub(bp[l], cscale(nbp, n[l]));
    const cx<T> uT = cscale(cadd(cscale(buT, c), mul_i(cscale(nxp[l], ks2))), iD);
    const cx<T> pT = cscale(cadd(mul_i(cscale(nxu[l], ks2)), cscale(bpT, a)), iD);
    u[l] = cadd(uT, cscale(nbu, n[l] * iL));
    ph[l] = cadd(pT, cscale(nbp, n[l] * iP));
  }
  green_strains<T>(xi, u, ph, scale, tau, mu);
}

// General reference medium (Eq. 5 tensors A0_klmn, B0_lkmn).  Writing
// phi = i psi turns K into the real symmetric positive definite matrix
//   S = [[A0_alkj xi_a xi_k,  xi_a C_alj],
//        [xi_a C_ajl,         B0_lkjn xi_k xi_n - F_lj]],
//   C_abj = A0_abkl eps_lkj,  F_lj = eps_lkm C_kmj,
// and the system into S (u, psi) = (bu, -i bp).  Each of the 21 upper
// entries of S (row by row) is a polynomial in xi; G holds its 10
// coefficients of xi1^2, xi2^2, xi3^2, xi1 xi2, xi1 xi3, xi2 xi3, xi1, xi2,
// xi3, 1.  S is factored as L D L^T (no pivoting: S is positive definite),
// and the real and imaginary parts of the sources are its two right-hand
// sides.
constexpr int kSymEntries = 21;
constexpr int kSymCoef = 10;

template <class T>
__device__ __forceinline__ void green_apply_gen(const MP_GLOBAL double* G, T x1, T x2, T x3, T scale,
                                                cx<T>* tau /*9 in, e out*/, cx<T>* mu /*9 in, g out*/) {
  const T xi[3] = {x1, x2, x3};
  cx<T> b[6];
  {
    cx<T> bu[3], bp[3];
    green_sources<T>(xi, tau, mu, bu, bp);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      b[l] = bu[l];
      b[3 + l] = cx<T>{bp[l].im, -bp[l].re};   // -i bp
    }
  }
  const T mono[9] = {x1 * x1, x2 * x2, x3 * x3, x1 * x2, x1 * x3, x2 * x3, x1, x2, x3};
  // entry (i, j), i <= j, of S: the u-psi block is linear in xi, the u-u
  // block quadratic, the psi-psi block quadratic plus a constant (the other
  // coefficients of an entry are zero and not read)
  auto entry = [&](int i, int j) {
    const MP_GLOBAL double* g = G + kSymCoef * (i * (11 - i) / 2 + j);
    T v = T(0);
    if (i < 3 && j >= 3) {
#pragma unroll
      for (int m = 6; m < 9; ++m) v += T(g[m]) * mono[m];
    } else {
#pragma unroll
      for (int m = 0; m < 6; ++m) v += T(g[m]) * mono[m];
      if (i >= 3) v += T(g[9]);
    }
    return v;
  };
  // S = L D L^T column by column, each entry of S evaluated where it is
  // needed.  U = L D (below the diagonal) and 1/D are kept, which the
  // elimination and both triangular solves use as they are.
  T U[6][6], id[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T d = entry(j, j);
#pragma unroll
    for (int k = 0; k < j; ++k) d -= U[j][k] * U[j][k] * id[k];
    id[j] = T(1) / d;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      T v = entry(j, i);
#pragma unroll
      for (int k = 0; k < j; ++k) v -= U[i][k] * U[j][k] * id[k];
      U[i][j] = v;
    }
  }
  // w = D^-1 L^-1 b: w_i = (b_i - sum_k U_ik w_k) / d_i; then
  // x = L^-T w: x_i = w_i - (sum_k U_ki x_k) / d_i
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int k = 0; k < i; ++k) b[i] = csub(b[i], cscale(b[k], U[i][k]));
    b[i] = cscale(b[i], id[i]);
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    cx<T> r = {0, 0};
#pragma unroll
    for (int k = i + 1; k < 6; ++k) r = cadd(r, cscale(b[k], U[k][i]));
    b[i] = csub(b[i], cscale(r, id[i]));
  }
  const cx<T> u[3] = {b[0], b[1], b[2]};
  const cx<T> ph[3] = {mul_i(b[3]), mul_i(b[4]), mul_i(b[5])};   // phi = i psi
  green_strains<T>(xi, u, ph, scale, tau, mu);
}

// Index of entry (i, j), i <= j, of a symmetric 6 x 6 matrix stored as its
// upper triangle row by row (21 entries).
__host__ __device__ constexpr int sym6(int i, int j) { return i * (11 - i) / 2 + j; }

// The Green operator stored per frequency, as the paper precomputes it
// (Sec. 2.4): the inverse of the real symmetric symbol S(xi) of
// green_apply_gen (an isotropic reference medium enters through its Eq. 6
// tensors), out[sym6(i, j)] = (S^-1)_ij.  FP64, from the coefficients G;
// S = L D L^T as in green_apply_gen, then S^-1 column by column from the
// unit vectors.
__device__ inline void green_symbol_inverse(const MP_GLOBAL double* G, double x1, double x2, double x3,
                                            double* out) {
  const double mono[9] = {x1 * x1, x2 * x2, x3 * x3, x1 * x2, x1 * x3, x2 * x3, x1, x2, x3};
  double S[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      const MP_GLOBAL double* g = G + kSymCoef * sym6(i, j);
      double v = 0.0;
      for (int m = 0; m < 9; ++m) v += g[m] * mono[m];
      S[i][j] = S[j][i] = v + g[9];
    }
  double U[6][6], id[6];
  for (int j = 0; j < 6; ++j) {
    double d = S[j][j];
    for (int k = 0; k < j; ++k) d -= U[j][k] * U[j][k] * id[k];
    id[j] = 1.0 / d;
    for (int i = j + 1; i < 6; ++i) {
      double v = S[j][i];
      for (int k = 0; k < j; ++k) v -= U[i][k] * U[j][k] * id[k];
      U[i][j] = v;
    }
  }
  for (int c = 0; c < 6; ++c) {
    double b[6];
    for (int i = 0; i < 6; ++i) {
      b[i] = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) b[i] -= b[k] * U[i][k];
      b[i] *= id[i];
    }
    for (int i = 4; i >= 0; --i) {
      double r = 0.0;
      for (int k = i + 1; k < 6; ++k) r += b[k] * U[k][i];
      b[i] -= r * id[i];
    }
    for (int i = 0; i <= c; ++i) out[sym6(i, c)] = b[i];
  }
}

// Green operator at one frequency from its stored inverse symbol: entry e
// at Si[e * es].  (u, psi) = S^-1 (bu, -i bp), phi = i psi, as in
// green_apply_gen.
template <class T>
__device__ __forceinline__ void green_apply_stored(const MP_GLOBAL T* Si, long es, T x1, T x2, T x3, T scale,
                                                   cx<T>* tau /*9 in, e out*/, cx<T>* mu /*9 in, g out*/) {
  const T xi[3] = {x1, x2, x3};
  cx<T> b[6];
  {
    cx<T> bu[3], bp[3];
    green_sources<T>(xi, tau, mu, bu, bp);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      b[l] = bu[l];
      b[3 + l] = cx<T>{bp[l].im, -bp[l].re};   // -i bp
    }
  }
  cx<T> x[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = cx<T>{T(0), T(0)};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      const T v = Si[es * sym6(i, j)];
      x[i] = cadd(x[i], cscale(b[j], v));
      if (j != i) x[j] = cadd(x[j], cscale(b[i], v));
    }
  const cx<T> u[3] = {x[0], x[1], x[2]};
  const cx<T> ph[3] = {mul_i(x[3]), mul_i(x[4]), mul_i(x[5])};
  green_strains<T>(xi, u, ph, scale, tau, mu);
}

}  // namespace mp
