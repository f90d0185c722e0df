// Kernels of one fixed-point iteration of the micropolar basic scheme (Alg. 2)
// and of the step control around it.
//
// Layout in HBM (x fastest, voxel index (z n1 + y) n0 + x):
//   S      half spectra of the 18 components, component-interleaved:
//          [kz][ky][kx][c], kx < n0/2 (the x-Nyquist bin is dropped: the
//          Green operator zeroes it), complex T.  A spectral row (kz, ky) is
//          one contiguous run of n0/2 * 18 values; a y or z tile of TX
//          consecutive kx is a contiguous run of TX * 18 values per point.
//   E      current strain e (c = 0..8) and curvature gamma (c = 9..17), SoA,
//          FP64 in both precisions
//   Eprev  the same fields one converged step earlier (extrapolation), FP64
//   base   history base t_n - A e_n (0..8), m_n - B gamma_n (9..17), T
//   pq     p_n, q_n of the last committed step, FP64
//
// One loop iteration: Y_FWD -> Z_GREEN (z forward, Green operator, z
// inverse) -> Y_INV -> x pass ITER (x inverse, + E / Gamma, Alg. 1, error
// partials, polarization, x forward) -> error rows -> error measure.
// Between two load steps a single x pass TRANS commits the converged step
// (final return map, new history base, output fields, step averages) and
// opens the next one (extrapolated first iterate, its return map and
// polarization, x forward).
//
// Every pass is written as a per-tile device function.  The single-RVE
// kernels map one tile to one block; the resident-batch kernels run the same
// functions from a persistent grid over work lists, so a batched RVE takes
// bit-for-bit the same arithmetic as when it is solved alone.
#pragma once

#include "device_math.hpp"

namespace mp {

constexpr int kLev = 15;          // per-level error partials
constexpr int kNPart = 2 * kLev;  // error partial rows of an ITER x pass
constexpr int kNAvg = 40;         // step-average rows of a TRANS x pass
constexpr int kRed = 32;          // per-wave LDS reduction slots

struct Ctl {
  int done;       // 0 running, 1 converged / fixed count reached, 2 max_iter, 3 diverged
  int iters;      // loop iterations of the current step
  int fixed;      // > 0: run exactly this many iterations
  int max_iter;
  double err;
  double tol;
  int norm;       // 0 local (Eq. 38), 1 average (Eq. 37)
  int best_it;    // iteration that set `best`
  double err_parts[4];
  double best;    // smallest err of the step so far (divergence test)
  // low precision: the spectrum the next x pass reads carries the whole
  // polarization (0) or its increment (1); the pass writes the next one as
  // wr_incr says
  int rd_incr;
  int wr_incr;
};

// Low precision: a step starts with whole-polarization iterations and turns
// to increments once the error measure is below this, or has not improved
// for kIncrStall iterations (the rounding floor of the whole form).
constexpr double kIncrFrom = 1e-3;
constexpr int kIncrStall = 20;

enum XMode { X_ITER = 0, X_TRANS = 1, X_FWD_ONLY = 2, X_INV_ONLY = 3 };
// Z_GREEN_AN: Z_GREEN with a general (Eq. 5) reference medium; Z_GREEN_ST:
// Z_GREEN with the Green operator read from its stored table
enum AMode { Y_FWD = 0, Y_INV = 1, Z_GREEN = 2, Z_FWD = 3, Z_GREEN_AN = 4, Z_GREEN_ST = 5 };

template <class T>
struct XArgs {
  long nrows;       // n1 * n2
  const cx<T>* tw;  // n0-entry twiddles
  cx<T>* S;
  long nvox;
  double* E;        // current iterate e (0..8), gamma (9..17): FP64 in both precisions
  double* Eprev;    // the same one committed step earlier (extrapolation)
  T* base;
  double* pq;
  T* out_tm;        // committed t (0..8), m (9..17)
  double* out_pq;   // committed p, q
  const uint8_t* phase;
  const PhaseC* params;
  double* partials; // [row][tile]
  RefC ref;
  double mac[18];   // E then Gamma of the step being opened / iterated
  double r;         // extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
  int first;        // TRANS: first step, start from the uniform mac
  int commit;       // TRANS: commit the converged state held in E
  int init;         // TRANS: open the next step
  int n_aniso;      // records in `aniso` (AN kernels)
  const T* fin;     // X_FWD_ONLY input (18 n)
  T* fout;          // X_INV_ONLY output (18 n)
  const T* eig;     // optional eigenstress (18 n): subtracted in every polarization
  double relax;     // augmented-Lagrangian ITER passes: over-relaxation of the compatible field
  int al;           // 1: this RVE's ITER passes run the augmented-Lagrangian scheme (batch
                    // kernels choose per RVE; a plan chooses its kernel instead)
  const double* aniso;  // Eq. 5 row matrices, [record][level][81] (AN kernels)
  const double* refan;  // row matrices [level][81] of a general reference medium
                        // (AN kernels), or null: the isotropic constants `ref`
};

// deterministic sum over a 64-lane wavefront (every lane gets the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// v of lane (this lane xor o), o a power of two below 64: lane distances 1,
// 2 and 8 by DPP moves (quad permutations, a rotation by 8 within each row
// of 16 lanes), 4 and 16 by LDS swizzles (xor masks within 32 lanes), 32 by
// a permute through LDS
__device__ __forceinline__ double xor_lanes(double v, int o) {
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
  const int lo = int(unsigned(bits)), hi = int(unsigned(bits >> 32));
  int a, b;
  switch (o) {
    case 1:
      a = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      b = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 2:
      a = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      b = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 8:
      a = __builtin_amdgcn_update_dpp(0, lo, 0x128, 0xF, 0xF, false);
      b = __builtin_amdgcn_update_dpp(0, hi, 0x128, 0xF, 0xF, false);
      break;
    case 4:
      a = __builtin_amdgcn_ds_swizzle(lo, 0x101F);
      b = __builtin_amdgcn_ds_swizzle(hi, 0x101F);
      break;
    case 16:
      a = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
      b = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
      break;
    default:
      return __shfl_xor(v, o, 64);
  }
  return __longlong_as_double(
      static_cast<long long>((static_cast<unsigned long long>(unsigned(b)) << 32) | unsigned(a)));
}

// NaN-propagating max (a non-finite field must not look converged)
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

// Deterministic reduce-scatter of K values (K a power of two, 2..16) over a
// 64-lane wavefront.  At each exchange (lane distance 32, 16, ...) a lane
// keeps one half of its remaining values and adds in its partner's copies of
// that half; the one value left is then completed over the lanes that share
// it.  Value j is a NaN-propagating maximum when bit j of maxmask is set,
// else a sum.  The first lane of each group writes its value to out[index].
// 16 values take 34 cross-lane moves instead of 6 per value.
template <int K>
__device__ __forceinline__ void wave_reduce(double (&v)[K], unsigned maxmask, int lane, double* out) {
  static_assert(K >= 2 && K <= 16 && (K & (K - 1)) == 0, "K = 2, 4, 8, 16");
  int base = 0;
#pragma unroll
  for (int o = 32, k = K / 2; k >= 1; o >>= 1, k >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < k; ++i) {
      const double send = up ? v[i] : v[i + k];
      const double keep = up ? v[i + k] : v[i];
      const double recv = xor_lanes(send, o);
      const int j = base + (up ? k : 0) + i;
      v[i] = ((maxmask >> j) & 1u) ? nmax(keep, recv) : keep + recv;
    }
    if (up) base += k;
  }
  const bool mx = (maxmask >> base) & 1u;
#pragma unroll
  for (int o = 32 / K; o > 0; o >>= 1) {
    const double recv = xor_lanes(v[0], o);
    v[0] = mx ? nmax(v[0], recv) : v[0] + recv;
  }
  if ((lane & (64 / K - 1)) == 0) out[base] = v[0];
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nmax(v, __shfl_xor(v, o, 64));
  return v;
}

// x-pass launch shape for a row length N0 in precision T: ROWS rows per tile
// (the last tile may be ragged), one lane per voxel and Alg. 1 level, each
// level padded to whole wavefronts.  The levels are independent through the
// whole pass (transforms, return map, error partials), so a block runs LPB
// of them: both (FP64 rows up to 128, the faster form there) or one, which
// halves the block's LDS (5 pencils per row instead of 10) and lets more
// blocks share a CU (FP64 rows of 256: three blocks per CU instead of one).
template <class T, int N0>
struct XShape {
  static constexpr int LPB = (sizeof(T) == 8 && N0 <= 128) ? 2 : 1;
  static constexpr int ROWS = N0 >= 128 ? 1 : 128 / N0;
  static constexpr int VPB = ROWS * N0;
  static constexpr int VPAD = (VPB + 63) / 64 * 64;
  static constexpr int NTHR = LPB * VPAD;
  static constexpr int NH = N0 / 2;
  static constexpr int NPK = 5 * LPB * ROWS;   // complex pencils held in LDS
};

// Block b of an x-pass grid -> (tile, first level).  With both levels in a
// block, block b is tile b.  With one, blocks b and b + 8 take the two levels
// of one tile: the chip deals consecutive blocks to its 8 XCDs in turn, so
// both run on one XCD at about the same time and the spectrum lines they
// share (the two levels' components interleave in one run per kx) are
// fetched into one L2 once.  Tiles >= ntiles (padding to a multiple of 8)
// have no work.
template <int LPB>
__device__ __forceinline__ void x_item(long b, long* tile, int* lvl0) {
  if (LPB == 2) {
    *lvl0 = 0;
    *tile = b;
  } else {
    *lvl0 = int((b >> 3) & 1);
    *tile = (b >> 4) * 8 + (b & 7);
  }
}
template <int LPB>
constexpr long x_grid(long ntiles) { return LPB == 2 ? ntiles : 2 * ((ntiles + 7) / 8 * 8); }

// Real fields packed two per complex pencil for the x transforms, only like
// with like: pencils 0-3 carry strain-like components 0-7 in pairs, pencil 4
// component 8 alone, pencils 5-8 curvature-like components 9-16 in pairs,
// pencil 9 component 17 alone.  (Unpacking a field from a pencil shared with
// a much larger one would cost it relative precision.)
constexpr int kPencils = 10;
__device__ __forceinline__ int pencil_of(int c) {
  return c < 8 ? (c >> 1) : c == 8 ? 4 : c < 17 ? 5 + ((c - 9) >> 1) : 9;
}
__device__ __forceinline__ int part_of(int c) {
  return c < 8 ? (c & 1) : (c == 8 || c == 17) ? 0 : ((c - 9) & 1);
}
__device__ __forceinline__ int pencil_re(int q) { return q < 5 ? 2 * q : 2 * q - 1; }
__device__ __forceinline__ int pencil_im(int q) { return (q == 4 || q == 9) ? -1 : pencil_re(q) + 1; }

// Row of the step-average record written by level L, slot j < 20 of a TRANS
// pass: <t> or <m> (0..17), <e> or <gamma> (18..35), <p> or <q> (36, 37),
// <t_eq> or <m_eq> (38, 39).
__device__ __forceinline__ int avg_row(int L, int j) {
  return j < 9 ? L * 9 + j : j < 18 ? 18 + L * 9 + (j - 9) : j == 18 ? 36 + L : 38 + L;
}

// x pass over levels [lvl0, lvl0 + LPB) of one tile of ROWS rows of N0
// voxels: level 0 the macro level of Alg. 1 (e -> t, tau; components 0..8),
// level 1 the micro level (gamma -> m, mu; components 9..17), each level's 9
// fields held in LDS as 5 complex pencils per row (two real transforms in one
// complex transform).  Lanes [0, VPAD) run level lvl0, lanes [VPAD, 2 VPAD)
// level lvl0 + 1 when the block has both: the level is uniform over each
// wavefront.
// Each lane prefetches its old strain, history base and p_n / q_n before the
// transforms so the loads overlap them.
//   lds, lds2: NPK * N0 complex each (the x transforms ping-pong between
//   them, one barrier per stage);  red: NTHR / 64 rows of kRed doubles;  tw:
//   the N0-entry twiddle table in LDS;  tid: the thread index.
//   AN: some phases have the general tensors of Eq. 5 (elastic phases: their
//   stresses are the elastic law from the history base, no return map).
//   ALG (ITER, FP64): an iteration of the augmented-Lagrangian scheme in
//   place of the basic one.  E holds the local strain d, and the spectrum
//   the Green operator's response to the polarization s(d) - C0 d; the pass
//   forms the compatible field e = E + that response, over-relaxes it (e^ =
//   w e + (1 - w) d_old), solves the local step s(d) + C0 d = s(d_old) +
//   C0 e^ (al_macro_local, al_micro_local), and goes on with d as the new
//   iterate (return map, error measure and polarization as in the basic pass).
//   rd_incr, wr_incr (ITER, low precision only): in low precision (T =
//   float) the strain state, the return map and the polarization stay FP64
//   and only the transforms run in T.  A step opens (TRANS) with the whole
//   polarization of its first iterate; an ITER pass reads a spectrum of the
//   whole polarization (rd_incr = 0: e = E + G tau) or of its increment
//   (rd_incr = 1: e = e_old + G (tau_i - tau_{i-1}), the Green operator being
//   linear), and writes the whole polarization or the increment
//   (wr_incr).  The loop control turns a step to increments once the error
//   measure is small: then the transforms' rounding scales with the
//   increment, not with the field, and the step reaches its tolerance.
//   stash: LDS of 9 * NTHR doubles for low-precision ITER passes (unused
//   otherwise), lane-private slots c * NTHR + tid.
template <class T, int MODE, int N0, bool AN = false, bool ALG = false>
__device__ __forceinline__ void xpass_tile(const XArgs<T>& a, long tile, int lvl0, int ntiles, cx<T>* lds,
                                           cx<T>* lds2, double (*red)[kRed], const cx<T>* tw, int tid,
                                           bool rd_incr, bool wr_incr, double* stash) {
  using X = XShape<T, N0>;
  constexpr int ROWS = X::ROWS, VPB = X::VPB, VPAD = X::VPAD, NTHR = X::NTHR, NH = X::NH;
  constexpr int NPK = X::NPK;
  // buffer holding the spatial-domain pencils after the inverse transform,
  // and the buffer holding the spectra after the forward transform
  constexpr bool ODD = fft_pp_stages<N0>() % 2 == 1;
  constexpr bool SP2 = (MODE == X_ITER || MODE == X_INV_ONLY) && ODD;
  cx<T>* const sp = SP2 ? lds2 : lds;
  cx<T>* const other = SP2 ? lds : lds2;
  cx<T>* const fq = ODD ? other : sp;
  T* ldr = reinterpret_cast<T*>(sp);
  constexpr int KP = kPencils / 2;     // pencils of one level
  constexpr int KPB = KP * X::LPB;     // pencils of the block's levels, per row
  const long row0 = tile * ROWS;
  // (both levels in the block: lvl0 = 0)
  const int lvl = X::LPB == 2 ? __builtin_amdgcn_readfirstlane(tid >= VPAD ? 1 : 0) : lvl0;
  const int v = tid - (lvl - lvl0) * VPAD;
  const int vr = v < VPB ? v / N0 : 0, vx = v < VPB ? v % N0 : 0;
  const bool own = v < VPB && row0 + vr < a.nrows;
  // 32-bit voxel offset into wave-uniform component bases (at most 2^24 voxels)
  const int gi = own ? int((row0 + vr) * N0 + vx) : 0;
  const long nv = a.nvox;
  MP_GLOBAL cx<T>* const S = glob(a.S);
  MP_GLOBAL double* const Elv = glob(a.E) + (long)lvl * 9 * nv;
  MP_GLOBAL double* const Eprev = glob(a.Eprev);
  MP_GLOBAL T* const Blv = glob(a.base) + (long)lvl * 9 * nv;
  MP_GLOBAL double* const pq = glob(a.pq);
  MP_GLOBAL double* const partials = glob(a.partials);
  const int rows_here = int(a.nrows - row0 < ROWS ? a.nrows - row0 : ROWS);

  // prefetch this lane's history (ITER, TRANS); the return map, the
  // polarization and the error measure run in FP64 in both precisions.  The
  // strain state and the base are read once per pass: non-temporal loads keep
  // them from displacing the spectrum in the caches (128^3 FP64: x pass 0.330
  // against 0.342 ms)
  double eo[9], bb[9];
  double hn = 0.0;
  int ph = 0;
#pragma unroll
  for (int c = 0; c < 9; ++c) eo[c] = bb[c] = 0.0;
  if ((MODE == X_ITER || MODE == X_TRANS) && own) {
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      eo[c] = __builtin_nontemporal_load(&Elv[c * nv + gi]);
      bb[c] = double(__builtin_nontemporal_load(&Blv[c * nv + gi]));
    }
    hn = pq[lvl * nv + gi];
    ph = glob(a.phase)[gi];
  }

  if (MODE == X_ITER || MODE == X_INV_ONLY) {
    // half spectra -> packed full spectra Z = A + i B, Z(n0 - k) = conj A + i conj B
    const int items = rows_here * NH * KPB;
    auto get = [&](int w, cx<T>& A, cx<T>& B) {
      const int r = w / (NH * KPB), rem = w % (NH * KPB);
      const int kx = rem / KPB, q = lvl0 * KP + rem % KPB;
      const MP_GLOBAL cx<T>* srow = S + (row0 + r) * (NH * 18) + kx * 18;
      const int cim = pencil_im(q);
      A = gload(srow + pencil_re(q));
      B = cx<T>{T(0), T(0)};
      if (cim >= 0) B = gload(srow + cim);
    };
    auto put = [&](int w, cx<T> A, cx<T> B) {
      const int r = w / (NH * KPB), rem = w % (NH * KPB);
      const int kx = rem / KPB, ql = rem % KPB;
      cx<T>* pen = lds + (r * KPB + ql) * N0;
      pen[kx] = cx<T>{A.re - B.im, A.im + B.re};
      if (kx > 0)
        pen[N0 - kx] = cx<T>{A.re + B.im, B.re - A.im};
      else
        pen[NH] = cx<T>{T(0), T(0)};
    };
    if constexpr (sizeof(T) == 8) {
      // FP64: every load of the thread is issued before the first is waited
      // for (measured faster; in FP32 the streaming loop below is faster)
      constexpr int MBX = (ROWS * NH * KPB + NTHR - 1) / NTHR;
      cx<T> A[MBX], B[MBX];
#pragma unroll
      for (int j = 0; j < MBX; ++j)
        if (tid + j * NTHR < items) get(tid + j * NTHR, A[j], B[j]);
#pragma unroll
      for (int j = 0; j < MBX; ++j)
        if (tid + j * NTHR < items) put(tid + j * NTHR, A[j], B[j]);
    } else {
      for (int w = tid; w < items; w += NTHR) {
        cx<T> A, B;
        get(w, A, B);
        put(w, A, B);
      }
    }
    __syncthreads();
    fft_pp<T, true, N0, 1, NPK, 1, N0, false, NTHR>(lds, lds2, tw, tid);
  }

  // LDS scalar slot of field c (0..17, of the block's levels) of this lane's voxel
  auto slot = [&](int c) { return 2 * ((vr * KPB + pencil_of(c) - lvl0 * KP) * N0 + vx) + part_of(c); };

  if (MODE == X_INV_ONLY) {
    if (own)
#pragma unroll
      for (int c = 0; c < 9; ++c) glob(a.fout)[(lvl * 9 + c) * nv + gi] = ldr[slot(lvl * 9 + c)];
    return;
  }

  // Per-wave partial sums (or maxima) by a reduce-scatter over the
  // wavefront (fixed order), then over the waves of a level in order.
  const int lane = tid & 63, wv = tid >> 6;

  // this lane's half of the phase record.  Low-precision loop iterations
  // read it again at each return map instead (two per voxel): held across
  // the pass, its eight doubles made the pass spill at 3 waves per SIMD
  // (256^3 mixed: 2.72 ms with the record held, 2.48 ms read twice)
  constexpr bool REREAD = sizeof(T) < sizeof(double) && MODE == X_ITER;
  MacroC ct;
  MicroC cm;
  if (MODE != X_FWD_ONLY && !REREAD) {
    if (lvl == 0)
      ct = gread(&glob(a.params)[ph].t);
    else
      cm = gread(&glob(a.params)[ph].m);
  }
  // the record's address, opaque to the compiler so that the two reads are
  // not merged into one held value
  auto record = [&]() {
    const MP_GLOBAL PhaseC* pp = glob(a.params) + ph;
    asm volatile("" : "+v"(pp));
    return pp;
  };
  // this lane's Eq. 5 record (AN kernels), -1 for an Eq. 6 phase
  int aid = -1;
  if (AN && MODE != X_FWD_ONLY) aid = int(glob(&a.params[ph].t.aid)[0]);

  if (MODE == X_TRANS && a.commit) {
    // commit (end of the step loop): final return map at the converged
    // iterate, new history base, output fields, step-average partials
    double tc[9];
    double pc = 0.0, eq = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) tc[c] = 0.0;
    if (own) {
      double r0[9];
      if (AN && aid >= 0) {
        aniso_apply_wave<double>(a.aniso, a.n_aniso, aid, lvl, eo, r0);
#pragma unroll
        for (int c = 0; c < 9; ++c) tc[c] = r0[c] + bb[c];
        pc = hn;
        eq = lvl == 0 ? macro_equivalent<double>(ct, tc) : micro_equivalent<double>(cm, tc);
      } else if (lvl == 0) {
        macro_return<double>(ct, eo, bb, hn, tc, pc);
        apply_A<double>(ct.lam, ct.mu, ct.kap, eo, r0);
        eq = macro_equivalent<double>(ct, tc);
      } else {
        micro_return<double>(cm, eo, bb, hn, tc, pc);
        apply_B<double>(cm.alp, cm.bet, cm.gam, eo, r0);
        eq = micro_equivalent<double>(cm, tc);
      }
      MP_GLOBAL T* const Olv = glob(a.out_tm) + (long)lvl * 9 * nv;
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        // the base as stored (rounded to T), also for the next step's
        // first return map below
        const T b = T(tc[c] - r0[c]);
        bb[c] = double(b);
        Blv[c * nv + gi] = b;
        Olv[c * nv + gi] = T(tc[c]);
      }
      hn = pc;
      pq[lvl * nv + gi] = pc;
      glob(a.out_pq)[lvl * nv + gi] = pc;
    }
    {
      double v[16];
#pragma unroll
      for (int c = 0; c < 9; ++c) v[c] = own ? double(tc[c]) : 0.0;
#pragma unroll
      for (int c = 0; c < 7; ++c) v[9 + c] = own ? double(eo[c]) : 0.0;
      wave_reduce<16>(v, 0u, lane, red[wv]);
      double w[4] = {own ? double(eo[7]) : 0.0, own ? double(eo[8]) : 0.0, own ? pc : 0.0,
                     own ? eq : 0.0};
      wave_reduce<4>(w, 0u, lane, red[wv] + 16);
    }
    __syncthreads();
    if (tid < X::LPB * kNAvg / 2) {   // 20 rows per level, its waves in order
      const int L = lvl0 + tid / 20, j = tid % 20;
      const int w0 = (L - lvl0) * (VPAD / 64), w1 = w0 + VPAD / 64;
      double y = red[w0][j];
      for (int w = w0 + 1; w < w1; ++w) y += red[w][j];
      partials[(long)avg_row(L, j) * ntiles + tile] = y;
    }
    if (!a.init) return;   // uniform over the block
  }

  {
    double e[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) e[c] = 0.0;
    if (own) {
      if (MODE == X_FWD_ONLY) {
#pragma unroll
        for (int c = 0; c < 9; ++c) e[c] = double(glob(a.fin)[(lvl * 9 + c) * nv + gi]);
      } else if (MODE == X_ITER) {
        if (sizeof(T) == 8 || !rd_incr) {
          // e = E + the fluctuation the Green operator returned (Alg. 2)
#pragma unroll
          for (int c = 0; c < 9; ++c) e[c] = double(ldr[slot(lvl * 9 + c)]) + a.mac[lvl * 9 + c];
        } else {
          // low precision: the transforms carried the polarization
          // increment, e = e_old + G(tau_i - tau_{i-1}) (the Green operator
          // is linear), so their rounding scales with the increment, not
          // with the field
#pragma unroll
          for (int c = 0; c < 9; ++c) e[c] = eo[c] + double(ldr[slot(lvl * 9 + c)]);
        }
      } else {  // X_TRANS: first iterate of the step (Alg. 2)
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const long at = (lvl * 9 + c) * nv + gi;
          const double old = Eprev[at];
          e[c] = a.first ? a.mac[lvl * 9 + c] : eo[c] + a.r * (eo[c] - old);
          Eprev[at] = eo[c];
        }
      }
    }
    // the single-field pencil of this level (4 or 9) has no imaginary field:
    // clear it, the transform must not read stale LDS
    if (own) ldr[2 * ((vr * KPB + (lvl - lvl0) * KP + KP - 1) * N0 + vx) + 1] = T(0);
    if (MODE == X_FWD_ONLY) {
      if (own)
#pragma unroll
        for (int c = 0; c < 9; ++c) ldr[slot(lvl * 9 + c)] = T(e[c]);
    } else {
      // stresses of a strain by this lane's law: Alg. 1 from the history
      // base, or the elastic law of an Eq. 5 phase
      auto law = [&](const double* x, double* out, double& pout) {
        if (AN && aid >= 0) {
          aniso_apply_wave<double>(a.aniso, a.n_aniso, aid, lvl, x, out);
#pragma unroll
          for (int c = 0; c < 9; ++c) out[c] += bb[c];
          pout = hn;
        } else if (lvl == 0) {
          macro_return<double>(REREAD ? gread(&record()->t) : ct, x, bb, hn, out, pout);
        } else {
          micro_return<double>(REREAD ? gread(&record()->m) : cm, x, bb, hn, out, pout);
        }
      };
      // the reference medium's stresses A0 e (B0 gamma) of the polarization
      auto ref_law = [&](const double* x, double* out) {
        if (AN && a.refan)
          aniso_apply<double>(cnst(a.refan) + lvl * 81, x, out);
        else if (lvl == 0)
          apply_A<double>(a.ref.lam, a.ref.mu, a.ref.kap, x, out);
        else
          apply_B<double>(a.ref.alp, a.ref.bet, a.ref.gam, x, out);
      };
      // low-precision loop iterations evaluate the old iterate's
      // polarization tau(e_old) first and park it in LDS (nine doubles per
      // lane, off the register file): the increment tau(e) - tau(e_old) and
      // the stress change of Eq. 37, sigma(e) - sigma(e_old) = that increment
      // + C0 (e - e_old), both come from it.  The FP64 pass recomputes
      // sigma(e_old) after the update, for the error measure only
      constexpr bool LOWP = sizeof(T) < sizeof(double) && MODE == X_ITER;
      double t[9], to[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) t[c] = to[c] = 0.0;
      double pnew, db_low = 0.0;
      if (own) {
        if constexpr (LOWP) {
          double pold, q0[9];
          law(eo, to, pold);
          ref_law(eo, q0);
#pragma unroll
          for (int c = 0; c < 9; ++c) stash[c * NTHR + tid] = to[c] - q0[c];
        }
        if constexpr (ALG) {
          // e holds the compatible field: the local step turns it into d
          double pold, eh[9], rr[9];
          law(eo, to, pold);
#pragma unroll
          for (int c = 0; c < 9; ++c) eh[c] = a.relax * e[c] + (1.0 - a.relax) * eo[c];
          ref_law(eh, rr);
#pragma unroll
          for (int c = 0; c < 9; ++c) rr[c] += to[c];
          if (lvl == 0)
            al_macro_local(ct, a.ref, rr, bb, hn, e);
          else
            al_micro_local(cm, a.ref, rr, bb, eh, hn, e);
          // the stresses of the new local strain follow from the equation
          // the local step solved, sigma(d) + C0 d = r: no second return map
          double c0d[9];
          ref_law(e, c0d);
#pragma unroll
          for (int c = 0; c < 9; ++c) t[c] = rr[c] - c0d[c];
        } else {
          law(e, t, pnew);
        }
        // polarization (Eq. 34): tau = t - A0 e ; mu = m - B0 gamma, less the
        // eigenstress when one is set (the manufactured stresses of the code
        // verification, App. D.1)
        double r0[9];
        ref_law(e, r0);
#pragma unroll
        for (int c = 0; c < 9; ++c) r0[c] = t[c] - r0[c];
        bool whole = true;
        if constexpr (LOWP) {
          double dt[9], de[9], q0[9];
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            dt[c] = r0[c] - stash[c * NTHR + tid];
            de[c] = e[c] - eo[c];
          }
          ref_law(de, q0);
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const double y = dt[c] + q0[c];
            db_low += y * y;
          }
          if (wr_incr) {
#pragma unroll
            for (int c = 0; c < 9; ++c) r0[c] = dt[c];
            whole = false;
          }
        }
        if (whole && a.eig) {
          const MP_GLOBAL T* const eg = glob(a.eig) + (long)lvl * 9 * nv;
#pragma unroll
          for (int c = 0; c < 9; ++c) r0[c] -= double(eg[c * nv + gi]);
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          ldr[slot(lvl * 9 + c)] = T(r0[c]);
          Elv[c * nv + gi] = e[c];
        }
      }
      if (MODE == X_ITER) {
        // error partials |da|, |db| (max), |da|, |db| (sum), |a|^2, |b|^2,
        // b (sum) with (a, b) = (e, t) on the macro level and (gamma, m) on
        // the micro level
        double da = 0, sa = 0, sb = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const double x = e[c] - eo[c];
          da += x * x;
          sa += e[c] * e[c];
          sb += t[c] * t[c];
        }
        da = sqrt(da);
        {
          // slots 0 (max) and 2 (sum) |da|, 4 |a|^2, 5 |b|^2, 6..14 b;
          // 1 and 3 (|db|) follow below into slots 16, 17
          double v[16];
          v[0] = own ? da : 0.0;
          v[1] = 0.0;
          v[2] = v[0];
          v[3] = 0.0;
          v[4] = own ? sa : 0.0;
          v[5] = own ? sb : 0.0;
#pragma unroll
          for (int c = 0; c < 9; ++c) v[6 + c] = own ? t[c] : 0.0;
          v[15] = 0.0;
          wave_reduce<16>(v, 0x1u, lane, red[wv]);
        }
        // the old iterate's stresses, recomputed from the old strain (Alg. 1)
        double db = db_low;
        if (own && !LOWP) {
          if constexpr (!LOWP && !ALG) {
            double pold;
            law(eo, to, pold);
          }
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const double y = t[c] - to[c];
            db += y * y;
          }
        }
        db = sqrt(db);
        {
          double w[2] = {own ? db : 0.0, own ? db : 0.0};
          wave_reduce<2>(w, 0x1u, lane, red[wv] + 16);
        }
        __syncthreads();
        if (tid < X::LPB * kLev) {   // kLev rows per level, its waves in order
          const int L = lvl0 + tid / kLev, j = tid % kLev;
          const int jj = j == 1 ? 16 : j == 3 ? 17 : j;
          const int w0 = (L - lvl0) * (VPAD / 64), w1 = w0 + VPAD / 64;
          double y = red[w0][jj];
          for (int w = w0 + 1; w < w1; ++w) y = (j < 2) ? nmax(y, red[w][jj]) : y + red[w][jj];
          partials[(long)(L * kLev + j) * ntiles + tile] = y;
        }
      }
    }
  }
  __syncthreads();
  fft_pp<T, false, N0, 1, NPK, 1, N0, false, NTHR>(sp, other, tw, tid);
  // unpack: A = (Z(k) + conj Z(-k)) / 2, B = (Z(k) - conj Z(-k)) / (2 i)
  for (int w = tid; w < rows_here * NH * KPB; w += NTHR) {
    const int r = w / (NH * KPB), rem = w % (NH * KPB);
    const int kx = rem / KPB, ql = rem % KPB, q = lvl0 * KP + ql;
    const cx<T>* pen = fq + (r * KPB + ql) * N0;
    const cx<T> zk = pen[kx];
    const cx<T> zm = pen[kx == 0 ? 0 : N0 - kx];
    MP_GLOBAL cx<T>* srow = S + (row0 + r) * (NH * 18) + kx * 18;
    const int cre = pencil_re(q), cim = pencil_im(q);
    gstore(srow + cre, cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)});
    if (cim >= 0) gstore(srow + cim, cx<T>{T(0.5) * (zk.im + zm.im), T(0.5) * (zm.re - zk.re)});
  }
}

// The ITER pass is held to 3 waves per SIMD (at most 168 VGPRs); its return
// map and polarization are FP64 in both precisions.  The augmented-Lagrangian
// ITER pass (a local solve per level on top) is held to 2 (256 VGPRs).
template <class T, int MODE, bool ALG = false>
constexpr int x_min_waves() { return MODE != X_ITER ? 1 : ALG ? 2 : 3; }

// the levels of one tile per block (x_item; grid x_grid(ntiles)); every
// kernel of the step loop returns at once when the step's control block says
// the loop is finished
template <class T, int MODE, int N0, bool AN = false, bool ALG = false>
__global__ void __launch_bounds__((XShape<T, N0>::NTHR), (x_min_waves<T, MODE, ALG>())) k_xpass(XArgs<T> a,
                                                                                       const Ctl* ctl,
                                                                                       int ntiles) {
  using X = XShape<T, N0>;
  if (ctl && ctl->done) return;
  // whole polarization or its increment (low precision, ITER)
  const bool rd = ctl && ctl->rd_incr, wr = ctl && ctl->wr_incr;
  __shared__ cx<T> lds[X::NPK * N0];
  __shared__ cx<T> lds2[X::NPK * N0];
  __shared__ double red[X::NTHR / 64][kRed];
  __shared__ cx<T> twl[N0];
  constexpr bool STASH = sizeof(T) < sizeof(double) && MODE == X_ITER;
  __shared__ double stash[STASH ? 9 * X::NTHR : 1];
  if constexpr (X::LPB == 2) {   // grid = ntiles, block b is tile b
    load_twiddles<T, N0, X::NTHR>(twl, glob(a.tw), threadIdx.x);
    xpass_tile<T, MODE, N0, AN, ALG>(a, blockIdx.x, 0, gridDim.x, lds, lds2, red, twl, threadIdx.x, rd, wr, stash);
  } else {
    long tile;
    int lvl;
    x_item<X::LPB>(blockIdx.x, &tile, &lvl);
    if (tile >= ntiles) return;
    load_twiddles<T, N0, X::NTHR>(twl, glob(a.tw), threadIdx.x);
    xpass_tile<T, MODE, N0, AN, ALG>(a, tile, lvl, ntiles, lds, lds2, red, twl, threadIdx.x, rd, wr, stash);
  }
}

// ---------------------------------------------------------------------------
// y and z passes over the interleaved half spectra.  A tile is TX
// consecutive kx at one kz (y pass) or one ky (z pass): L points x TX*18
// pencils, each point a contiguous run of TX*18 complex values.  Z_GREEN
// runs the forward z transform, the Green operator at every frequency of the
// tile (all 18 components are in LDS) and the inverse z transform, so the
// spectrum makes one HBM round trip for the three steps.
// ---------------------------------------------------------------------------
template <class T>
struct AxisArgs {
  cx<T>* S;
  long ostride;    // stride (complex) of the tile row index: kz for y, ky for z
  long pstride;    // stride (complex) between points of the transformed axis
  const cx<T>* tw;
  // Z_GREEN, Z_GREEN_AN, Z_GREEN_ST only
  int n0, n1, n2;
  double h, scale;
  RefC ref;
  const double* gsym;   // Z_GREEN_AN: symbol coefficients [21][10]
  const T* gtab;        // Z_GREEN_ST, and Z_GREEN_AN where set: the stored
                        // inverse symbol, [ky][kx][21][kz] (k_green_table)
};

template <int L, int TX>
struct AShape {
  static constexpr int NB = TX * 18;
  static constexpr int PTS = L * NB;
  static constexpr int NTHR = PTS > 2304 ? 512 : 256;
  static constexpr int MB = (PTS + NTHR - 1) / NTHR;   // values per thread of a tile
  static constexpr size_t LDS = size_t(PTS);   // complex values
};

// The thread index as a fresh value on every pass of a work loop: the
// per-thread index arithmetic of a pass then stays inside the loop instead of
// being hoisted out of it and held in registers across every item.
__device__ __forceinline__ int fresh_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Loads of tile (bx, by) into registers, MB values per thread.  All of a
// thread's loads are issued before the first is waited for; a loop that
// stores each value into LDS as it arrives keeps only one load in flight.
template <class T, int L, int TX>
__device__ __forceinline__ void axis_fetch(const AxisArgs<T>& a, int bx, int by,
                                           cx<T> (&v)[AShape<L, TX>::MB], int tid) {
  using A = AShape<L, TX>;
  const MP_GLOBAL cx<T>* g = glob(a.S) + (long)by * a.ostride + (long)bx * A::NB;
  const long ps = a.pstride;
#pragma unroll
  for (int j = 0; j < A::MB; ++j) {
    const int w = tid + j * A::NTHR;
    if (A::PTS % A::NTHR == 0 || w < A::PTS) v[j] = gload(g + (w / A::NB) * ps + w % A::NB);
  }
}

// How green_tile solves: the closed form of an isotropic reference medium,
// the factored symbol of a tensor one, or the stored inverse symbol
enum GKind { G_CLOSED = 0, G_FACTORED = 1, G_STORED = 2 };

// Green operator at frequency (kx, ky, kz) on its 18 components p[0..17]
// (in LDS): zero at the mean and at the y and z Nyquist indices
template <class T, int KIND>
__device__ __forceinline__ void green_freq(const AxisArgs<T>& a, int kx, int ky, int kz, cx<T>* p) {
  const bool zero = (kx == 0 && ky == 0 && kz == 0) || (2 * ky == a.n1) || (2 * kz == a.n2);
  if (zero) {
#pragma unroll
    for (int c = 0; c < 18; ++c) p[c] = cx<T>{T(0), T(0)};
  } else {
    cx<T> tau[9], mu[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      tau[c] = p[c];
      mu[c] = p[9 + c];
    }
    const double tp = 6.283185307179586476925286766559;
    const int my = (2 * ky < a.n1) ? ky : ky - a.n1;
    const int mz = (2 * kz < a.n2) ? kz : kz - a.n2;
    const T x1 = T(tp * kx / (a.n0 * a.h));
    const T x2 = T(tp * my / (a.n1 * a.h));
    const T x3 = T(tp * mz / (a.n2 * a.h));
    if constexpr (KIND == G_FACTORED) {
      green_apply_gen<T>(glob(a.gsym), x1, x2, x3, T(a.scale), tau, mu);
    } else if constexpr (KIND == G_STORED) {
      const long base = (long(ky) * (a.n0 / 2) + kx) * 21 * a.n2 + kz;
      green_apply_stored<T>(glob(a.gtab) + base, a.n2, x1, x2, x3, T(a.scale), tau, mu);
    } else {
      green_apply<T>(a.ref, x1, x2, x3, T(a.scale), tau, mu);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      p[c] = tau[c];
      p[9 + c] = mu[c];
    }
  }
}

// Green operator at the L * TX frequencies of z-pass tile (bx, by), in LDS
template <class T, int L, int TX, int KIND>
__device__ __forceinline__ void green_tile(const AxisArgs<T>& a, int bx, int by, cx<T>* lds, int tid) {
  using A = AShape<L, TX>;
  constexpr int NB = A::NB, NTHR = A::NTHR;
  for (int f = tid; f < L * TX; f += NTHR) {
    const int kz = f / TX, xl = f % TX;
    green_freq<T, KIND>(a, bx * TX + xl, by, kz, lds + kz * NB + xl * 18);
  }
}

// tile (bx, by): kx in [bx TX, bx TX + TX), kz = by (y pass) or ky = by (z
// pass); tw: the L-entry twiddle table in LDS.  The caller has synchronised
// the block since LDS was last read.
template <class T, int MODE, int L, int TX>
__device__ __forceinline__ void axis_tile(const AxisArgs<T>& a, int bx, int by, cx<T>* lds,
                                          const cx<T>* tw, int tid) {
  using A = AShape<L, TX>;
  constexpr int NB = A::NB, PTS = A::PTS, NTHR = A::NTHR;
  {
    cx<T> v[A::MB];
    axis_fetch<T, L, TX>(a, bx, by, v, tid);
#pragma unroll
    for (int j = 0; j < A::MB; ++j) {
      const int w = tid + j * NTHR;
      if (PTS % NTHR == 0 || w < PTS) lds[w] = v[j];
    }
  }
  __syncthreads();
  constexpr bool INV = MODE == Y_INV;
  fft_ct<T, INV, L, 1, NB, NB, 1, true, NTHR>(lds, tw, tid);
  if (MODE == Z_GREEN || MODE == Z_GREEN_AN || MODE == Z_GREEN_ST) {
    // Green operator at the L * TX frequencies of the tile.  Z_GREEN_AN also
    // serves a stored table (gtab set) and an isotropic reference (both
    // null): a batch class may hold every kind of RVE.  The choice is made
    // per tile, around the whole loop, so that the solves never share one
    // loop body's registers
    if (MODE == Z_GREEN_ST || (MODE == Z_GREEN_AN && a.gtab))
      green_tile<T, L, TX, G_STORED>(a, bx, by, lds, tid);
    else if (MODE == Z_GREEN_AN && a.gsym)
      green_tile<T, L, TX, G_FACTORED>(a, bx, by, lds, tid);
    else
      green_tile<T, L, TX, G_CLOSED>(a, bx, by, lds, tid);
    __syncthreads();
    fft_ct<T, true, L, 1, NB, NB, 1, true, NTHR>(lds, tw, tid);
  }
  MP_GLOBAL cx<T>* g = glob(a.S) + (long)by * a.ostride + (long)bx * NB;
  const long ps = a.pstride;
  // the general and stored Green steps need the registers that would
  // otherwise keep the load addresses alive for these stores: recompute them
  const int ts = MODE == Z_GREEN_AN || MODE == Z_GREEN_ST ? fresh_tid() : tid;
  for (int w = ts; w < PTS; w += NTHR) gstore(g + (w / NB) * ps + w % NB, lds[w]);
}

// XCD-aware tile order.  The chip hands consecutive blocks to its 8 XCDs in
// turn, and each XCD has its own L2.  A tile's runs (TX * 18 complex values
// per point) need not end on a cache line, so neighbouring tiles share lines:
// giving each XCD a contiguous range of tiles makes the shared lines hit in
// one L2 instead of being fetched once per XCD.  Maps block b of n to a tile.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = n / kXcd;
  return b < per * kXcd ? (b % kXcd) * per + b / kXcd : b;
}

// Waves per SIMD that the LDS tiles of a y / z pass allow (160 KB per CU),
// at most 4: the register budget then stays at 128 or more per lane.
template <class T, int L, int TX>
constexpr int axis_min_waves() {
  using A = AShape<L, TX>;
  const int bytes = int((A::LDS + L) * sizeof(cx<T>));
  const int blocks = (160 * 1024) / bytes;
  const int w = blocks * A::NTHR / 256;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// y or z pass of one cell: block b takes tile xcd_tile(b) of the gx * gy
// tiles (tile t = (t mod gx, t / gx)); the grid is one block per tile
template <class T, int MODE, int L, int TX>
__global__ void __launch_bounds__((AShape<L, TX>::NTHR), (axis_min_waves<T, L, TX>()))
    k_axis(AxisArgs<T> a, const Ctl* ctl, int gx) {
  if (ctl && ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  __shared__ cx<T> twl[L];
  load_twiddles<T, L, AShape<L, TX>::NTHR>(twl, glob(a.tw), threadIdx.x);
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  axis_tile<T, MODE, L, TX>(a, t % gx, t / gx, reinterpret_cast<cx<T>*>(smem_raw), twl, threadIdx.x);
}

// The stored Green operator (Sec. 2.4): the inverse symbol at every
// frequency of the half spectrum (kx < n0 / 2), from the symbol coefficients
// G, rounded to T, at tab[((ky nh + kx) 21 + e) n2 + kz] (nh = n0 / 2), so
// that a z-pass tile reads each entry as runs along kz.  Zero at the mean and
// at the y and z Nyquist indices, where the fluctuation is zero.  Grid-stride
// loop over the n2 n1 nh frequencies, kz fastest.
template <class T>
__global__ void __launch_bounds__(256) k_green_table(const double* G, int n0, int n1, int n2, double h, T* tab) {
  const int nh = n0 / 2;
  const long nf = long(n2) * n1 * nh;
  for (long f = long(blockIdx.x) * 256 + threadIdx.x; f < nf; f += long(gridDim.x) * 256) {
    const int kz = int(f % n2);
    const long r = f / n2;
    const int kx = int(r % nh), ky = int(r / nh);
    double v[21];
    if ((kx == 0 && ky == 0 && kz == 0) || 2 * ky == n1 || 2 * kz == n2) {
      for (int e = 0; e < 21; ++e) v[e] = 0.0;
    } else {
      const double tp = 6.283185307179586476925286766559;
      const int my = (2 * ky < n1) ? ky : ky - n1;
      const int mz = (2 * kz < n2) ? kz : kz - n2;
      green_symbol_inverse(glob(G), tp * kx / (n0 * h), tp * my / (n1 * h), tp * mz / (n2 * h), v);
    }
    MP_GLOBAL T* o = glob(tab) + (long(ky) * nh + kx) * 21 * n2 + kz;
    for (int e = 0; e < 21; ++e) o[long(e) * n2] = T(v[e]);
  }
}

// ---------------------------------------------------------------------------
// reductions and step control
// ---------------------------------------------------------------------------
// Deterministic reduction of one partial row over nblk tiles by a block of
// 256 threads (fixed order: two strided accumulators per thread, wave
// butterflies, then the four waves).  The result is valid in thread 0.
__device__ __forceinline__ double row_reduce(const MP_GLOBAL double* row, int nblk, bool mx,
                                             double* red4) {
  const int tid = threadIdx.x;
  double v0 = 0.0, v1 = 0.0;
  int b = tid;
  // chunks of 2U values per thread, all loaded before they are combined (in
  // the same order as the loop below, which takes the rest)
  constexpr int U = 8;
  for (; b + 512 * (U - 1) + 256 < nblk; b += 512 * U) {
    double x[2 * U];
#pragma unroll
    for (int k = 0; k < 2 * U; ++k) x[k] = row[b + 256 * k];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      v0 = mx ? nmax(v0, x[2 * k]) : v0 + x[2 * k];
      v1 = mx ? nmax(v1, x[2 * k + 1]) : v1 + x[2 * k + 1];
    }
  }
  for (; b + 256 < nblk; b += 512) {
    const double x = row[b], y = row[b + 256];
    v0 = mx ? nmax(v0, x) : v0 + x;
    v1 = mx ? nmax(v1, y) : v1 + y;
  }
  if (b < nblk) v0 = mx ? nmax(v0, row[b]) : v0 + row[b];
  double v = mx ? nmax(v0, v1) : v0 + v1;
  v = mx ? wave_max(v) : wave_sum(v);
  if ((tid & 63) == 0) red4[tid >> 6] = v;
  __syncthreads();
  return mx ? nmax(nmax(red4[0], red4[1]), nmax(red4[2], red4[3]))
            : ((red4[0] + red4[1]) + (red4[2] + red4[3]));
}

// row_reduce's result for nblk <= 64, from one wavefront: there the values
// sit in the lanes of the first wave, and the other three waves contribute
// +0 (sums) or nmax(0, 0) = 0 (maxima), so the same operations in the same
// order give the same value bit for bit.  x: this lane's value (lane < nblk).
// The result is valid in lane 0.
__device__ __forceinline__ double row_reduce_wave(double x, int lane, int nblk, bool mx) {
  double v0 = 0.0;
  const double v1 = 0.0, z = 0.0;
  if (lane < nblk) v0 = mx ? nmax(v0, x) : v0 + x;
  double v = mx ? nmax(v0, v1) : v0 + v1;
  v = mx ? wave_max(v) : wave_sum(v);
  return mx ? nmax(nmax(v, z), nmax(z, z)) : ((v + z) + (z + z));
}

// rows that hold maxima in an ITER x pass's error partials
__device__ __forceinline__ bool err_row_is_max(int j) { return (j % kLev) < 2; }

// error measure (Eqs. 36-38) from the reduced rows, and the step decision.
// <e> = E and <gamma> = Gamma hold exactly (the Green operator leaves no
// k = 0 fluctuation), so the averages of the strain-like fields are the
// prescribed ones.
__device__ __forceinline__ void err_finalize(const double* tot, long nvox, Ctl* ctl, const double* mac) {
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
        const double mc = b == 0 ? mac[L * 9 + c] : P[6 + c] * inv;
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
  if (err < ctl->best) {
    ctl->best = err;
    ctl->best_it = it;
  }
  // the x pass that follows reads what the last one wrote
  ctl->rd_incr = ctl->wr_incr;
  if (!ctl->wr_incr && (err <= kIncrFrom || it - ctl->best_it >= kIncrStall)) ctl->wr_incr = 1;
  // divergence: a non-finite measure, or growth far above the step's best
  // (a large err alone is legitimate when a field's mean is nearly zero)
  const bool diverged = !(err <= 1e300) || (it > 5 && err > 1e6 * ctl->best);
  int done = 0;
  if (diverged) {
    done = 3;
  } else if (ctl->fixed > 0) {
    if (it >= ctl->fixed) done = 1;
  } else if (err <= ctl->tol) {
    done = 1;
  } else if (it >= ctl->max_iter) {
    done = 2;
  }
  ctl->done = done;
}

struct ErrMacro {
  double v[18];   // prescribed E then Gamma of the step
};

__device__ __forceinline__ void ctl_reset(Ctl* ctl, int fixed, int max_iter, double tol, int norm) {
  ctl->done = 0;
  ctl->iters = 0;
  ctl->fixed = fixed;
  ctl->max_iter = max_iter;
  ctl->err = 2.0 * tol;
  ctl->tol = tol;
  ctl->norm = norm;
  ctl->best = 1e300;
  ctl->best_it = 0;
  ctl->rd_incr = 0;
  ctl->wr_incr = 0;
}

// widen n values to FP64 (field read-back into device memory)
template <class S>
__global__ void __launch_bounds__(256) k_widen(const S* in, double* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = double(in[i]);
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
