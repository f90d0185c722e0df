// Host-side helpers shared by the single-RVE plan and the resident batch:
// problem validation, workspace layout, per-phase constants, twiddles,
// reference medium and the compile-time size dispatch of the kernels.
#pragma once

#include "../../include/mp.h"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace mp {

inline thread_local std::string g_err;


inline mp_status fail(mp_status s, const std::string& msg) {
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

inline bool supported(int n) {
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

inline int x_rows(int n0) { return n0 >= 128 ? 1 : 128 / n0; }

// an: the problem has phases with Eq. 5 tensors (ITER and TRANS passes);
// al: augmented-Lagrangian iterations (FP64 ITER passes)
template <class T, int MODE>
void launch_x(int n0, int blocks, hipStream_t s, const XArgs<T>& a, const Ctl* ctl, bool an = false,
              bool al = false) {
  constexpr bool LAW = MODE == X_ITER || MODE == X_TRANS;
  constexpr bool ALX = MODE == X_ITER && sizeof(T) == sizeof(double);
  // blocks = row tiles; x_grid gives the blocks that run their levels
  switch (n0) {
#define MP_CASE(N)                                                                                    \
  case N: {                                                                                           \
    using X = XShape<T, N>;                                                                           \
    const dim3 grid(unsigned(x_grid<X::LPB>(blocks)));                                                \
    if (LAW && an)                                                                                    \
      hipLaunchKernelGGL((k_xpass<T, MODE, N, LAW>), grid, dim3(X::NTHR), 0, s, a, ctl, blocks);       \
    else if (ALX && al)                                                                               \
      hipLaunchKernelGGL((k_xpass<T, MODE, N, false, ALX>), grid, dim3(X::NTHR), 0, s, a, ctl, blocks); \
    else                                                                                              \
      hipLaunchKernelGGL((k_xpass<T, MODE, N>), grid, dim3(X::NTHR), 0, s, a, ctl, blocks);            \
    break;                                                                                            \
  }
    MP_SIZES(MP_CASE)
#undef MP_CASE
  }
}

template <class T, int MODE, int L, int TX>
void launch_axis_tx(int gx, int gy, hipStream_t s, const AxisArgs<T>& a, const Ctl* ctl) {
  const size_t shm = size_t(AShape<L, TX>::PTS) * sizeof(cx<T>);
  hipLaunchKernelGGL((k_axis<T, MODE, L, TX>), dim3(gx * gy), dim3(AShape<L, TX>::NTHR), shm, s, a, ctl,
                     gx);
}

// tiles: gx = n0 / 2 / tx along kx, gy along the other transverse axis
template <class T, int MODE>
void launch_axis(int L, int tx, int gx, int gy, hipStream_t s, const AxisArgs<T>& a, const Ctl* ctl) {
  switch (L) {
#define MP_CASE(N)                                                        \
  case N:                                                                 \
    if (tx == 1)                                                          \
      launch_axis_tx<T, MODE, N, 1>(gx, gy, s, a, ctl);                   \
    else                                                                  \
      launch_axis_tx<T, MODE, N, tx_wide(N)>(gx, gy, s, a, ctl);          \
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

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t S, E, Eprev, base, pq, out_tm, out_pq, phase, params, aniso, tw, partials, ctl, tot, gtab, total;
};

struct Geometry {
  int n0, n1, n2, nh;
  long nvox, nspec, nrows;
  int xblocks, txy, txz;
  int n_aniso;     // phases with Eq. 5 tensors
  int ref_tensor;  // 1: general reference medium of the phases' tensors (MP_REF_TENSOR_*)
  int green_stored;  // 1: the Green operator is stored per frequency (MP_GREEN_STORED)
};

// Doubles of the workspace's tensor table: the Eq. 5 row matrices of the
// anisotropic phases, then those of a general reference medium, then the
// reference's Fourier-symbol coefficients (with a tensor reference, or when
// the Green operator is stored).
inline size_t sym_offset(const Geometry& g) { return size_t(std::max(g.n_aniso + g.ref_tensor, 1)) * 162; }
inline size_t aniso_words(const Geometry& g) {
  return sym_offset(g) + (g.ref_tensor || g.green_stored ? size_t(kSymEntries) * kSymCoef : 0);
}
// Bytes of the stored Green operator: 21 words per frequency of the half
// spectrum
inline size_t green_table_bytes(const Geometry& g, size_t w) {
  return g.green_stored ? size_t(kSymEntries) * size_t(g.nspec) * w : 0;
}

// Symmetric positive definite 9 x 9 matrix (row-major), by Cholesky
inline bool spd9(const double* M) {
  double scale = 0.0;
  for (int i = 0; i < 81; ++i) {
    if (!std::isfinite(M[i])) return false;
    scale = std::max(scale, std::fabs(M[i]));
  }
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(M[9 * i + j] - M[9 * j + i]) > 1e-12 * scale) return false;
  double L[81] = {};
  for (int j = 0; j < 9; ++j) {
    double d = M[9 * j + j];
    for (int k = 0; k < j; ++k) d -= L[9 * j + k] * L[9 * j + k];
    if (!(d > 1e-14 * scale)) return false;
    L[9 * j + j] = std::sqrt(d);
    for (int i = j + 1; i < 9; ++i) {
      double v = M[9 * i + j];
      for (int k = 0; k < j; ++k) v -= L[9 * i + k] * L[9 * j + k];
      L[9 * i + j] = v / L[9 * j + j];
    }
  }
  return true;
}

// Row matrices of an Eq. 5 record: out[0..80] R with t_kl = R[3k + l][3m + n] e_mn
// (= A_klmn), out[81..161] with m_kl = R[3k + l][3m + n] gamma_mn (= B_lkmn)
inline void aniso_rows(const mp_aniso& a, double* out) {
  for (int i = 0; i < 81; ++i) out[i] = a.A[i];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l)
      for (int j = 0; j < 9; ++j) out[81 + 9 * (3 * k + l) + j] = a.B[9 * (3 * l + k) + j];
}

// Eq. 6 tensors of an isotropic phase in the storage orders of mp_aniso:
// A[27k + 9l + 3m + n] = A_klmn, B[27l + 9k + 3m + n] = B_lkmn.
inline void iso_tensors(const mp_phase& c, double* A, double* B) {
  auto d = [](int i, int j) { return i == j ? 1.0 : 0.0; };
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
          A[27 * k + 9 * l + 3 * m + n] = c.lambda * d(k, l) * d(m, n) + (c.mu + c.kappa) * d(k, m) * d(l, n) +
                                          (c.mu - c.kappa) * d(k, n) * d(l, m);
          B[27 * l + 9 * k + 3 * m + n] =
              c.alpha * d(k, l) * d(m, n) + c.beta * d(k, m) * d(l, n) + c.gamma * d(k, n) * d(l, m);
        }
}

// General reference medium, Alg. 2 taken literally: A0 = <A(x)>, B0 = <B(x)>
// over the cell with every phase's own tensors (Eq. 5 where the phase has
// them, else Eq. 6), in the storage orders of mp_aniso; with
// MP_REF_TENSOR_PHASE_MEAN the unweighted mean over the phases present.
inline mp_status reference_tensors(const mp_problem* prob, long nvox, mp_aniso* out) {
  std::vector<long> count(prob->n_phases, 0);
  for (long i = 0; i < nvox; ++i) count[prob->phase[i]]++;
  std::vector<const mp_aniso*> rec(prob->n_phases, nullptr);
  for (int j = 0; j < prob->n_aniso; ++j) rec[prob->aniso[j].phase] = &prob->aniso[j];
  int present = 0;
  for (int i = 0; i < prob->n_phases; ++i) present += count[i] ? 1 : 0;
  mp_aniso r{};
  r.phase = -1;
  for (int i = 0; i < prob->n_phases; ++i) {
    if (!count[i]) continue;
    double A[81], B[81];
    if (rec[i]) {
      std::memcpy(A, rec[i]->A, sizeof A);
      std::memcpy(B, rec[i]->B, sizeof B);
    } else {
      iso_tensors(prob->phases[i], A, B);
    }
    const double w = prob->ref_mode == MP_REF_TENSOR_PHASE_MEAN ? 1.0 / present
                                                                 : double(count[i]) / double(nvox);
    for (int k = 0; k < 81; ++k) {
      r.A[k] += w * A[k];
      r.B[k] += w * B[k];
    }
  }
  // <A> positive definite keeps the Fourier symbol positive definite at
  // every xi != 0 (no nonzero (u, phi) has e = 0), so <B> may be singular on
  // skew tensors (gamma = beta).  Valid phases give both; this is a guard.
  if (!spd9(r.A)) return fail(MP_E_INVALID, "reference tensor <A> is not positive definite over its index pairs");
  *out = r;
  return MP_OK;
}

// Sizes, x-pass tiles and y / z tile widths of an n0 x n1 x n2 grid (every
// n a supported length); no phases and no tensor reference
inline Geometry grid_geometry(int n0, int n1, int n2) {
  Geometry G{};
  G.n0 = n0; G.n1 = n1; G.n2 = n2; G.nh = n0 / 2;
  G.nvox = long(n0) * n1 * n2;
  G.nspec = long(n2) * n1 * G.nh;
  G.nrows = long(n1) * n2;
  const int rows = x_rows(n0);
  G.xblocks = int((G.nrows + rows - 1) / rows);
  G.txy = (G.nh % tx_wide(n1) == 0) ? tx_wide(n1) : 1;
  G.txz = (G.nh % tx_wide(n2) == 0) ? tx_wide(n2) : 1;
  return G;
}

inline mp_status reference_medium(const mp_problem* prob, long nvox, RefC* out);

inline mp_status validate(const mp_problem* p, Geometry* g) {
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
  if (p->ref_mode < 0 || p->ref_mode > 5) return fail(MP_E_INVALID, "ref_mode");
  if (p->scheme != MP_SCHEME_BASIC && p->scheme != MP_SCHEME_AL) return fail(MP_E_INVALID, "scheme");
  if (p->green_mode != MP_GREEN_COMPUTED && p->green_mode != MP_GREEN_STORED)
    return fail(MP_E_INVALID, "green_mode");
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
  if (p->n_aniso < 0 || p->n_aniso > p->n_phases) return fail(MP_E_INVALID, "n_aniso out of 0..n_phases");
  if (p->n_aniso > 0 && !p->aniso) return fail(MP_E_INVALID, "aniso is NULL");
  {
    std::vector<char> listed(size_t(p->n_phases), 0);
    for (int j = 0; j < p->n_aniso; ++j) {
      const mp_aniso& a = p->aniso[j];
      const std::string tag = "anisotropic record " + std::to_string(j) + ": ";
      if (a.phase < 0 || a.phase >= p->n_phases) return fail(MP_E_INVALID, tag + "phase id out of range");
      if (listed[a.phase]++) return fail(MP_E_INVALID, tag + "phase listed twice");
      const mp_phase& c = p->phases[a.phase];
      if (std::isfinite(c.tY) || std::isfinite(c.mY))
        return fail(MP_E_INVALID, tag + "the phase must be elastic (tY = mY = inf)");
      if (!spd9(a.A) || !spd9(a.B))
        return fail(MP_E_INVALID, tag + "A and B must be symmetric positive definite over their index pairs");
    }
  }
  const long nvox = long(p->n[0]) * p->n[1] * p->n[2];
  for (long i = 0; i < nvox; ++i)
    if (p->phase[i] >= p->n_phases) return fail(MP_E_INVALID, "phase id out of range");

  Geometry G = grid_geometry(p->n[0], p->n[1], p->n[2]);
  G.n_aniso = p->n_aniso;
  G.ref_tensor = p->ref_mode == MP_REF_TENSOR_MEAN || p->ref_mode == MP_REF_TENSOR_PHASE_MEAN ? 1 : 0;
  G.green_stored = p->green_mode == MP_GREEN_STORED ? 1 : 0;
  if (G.ref_tensor) {
    mp_aniso r;
    const mp_status rs = reference_tensors(p, nvox, &r);
    if (rs != MP_OK) return rs;
  }
  if (p->scheme == MP_SCHEME_AL) {
    if (p->precision != MP_FP64) return fail(MP_E_INVALID, "the augmented-Lagrangian scheme runs in FP64");
    if (p->n_aniso > 0 || G.ref_tensor)
      return fail(MP_E_INVALID, "the augmented-Lagrangian scheme takes Eq. 6 phases and an isotropic reference");
    if (!(p->relax > 0.0 && p->relax < 2.0)) return fail(MP_E_INVALID, "relax must lie in (0, 2)");
    RefC r;
    const mp_status rs = reference_medium(p, nvox, &r);
    if (rs != MP_OK) return rs;
    // the penalty must be positive definite on every part that carries
    // stress; the skew curvature carries none only where gamma = beta
    bool all_eq = true;
    std::vector<char> present(size_t(p->n_phases), 0);
    for (long i = 0; i < nvox; ++i) present[p->phase[i]] = 1;
    for (int i = 0; i < p->n_phases; ++i)
      if (present[i] && p->phases[i].gamma != p->phases[i].beta) all_eq = false;
    if (!(r.gam - r.bet > 0.0) && !all_eq)
      return fail(MP_E_INVALID, "the augmented-Lagrangian penalty needs gamma0 > beta0 unless every phase has "
                                "gamma = beta");
  }
  *g = G;
  return MP_OK;
}

inline Layout layout(const Geometry& g, size_t w /* bytes per bulk word */) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.S = take(18 * g.nspec * 2 * w);
  L.E = take(18 * g.nvox * sizeof(double));       // the strain state is FP64 in both precisions
  L.Eprev = take(18 * g.nvox * sizeof(double));
  L.base = take(18 * g.nvox * w);
  L.pq = take(2 * g.nvox * sizeof(double));
  L.out_tm = take(18 * g.nvox * w);
  L.out_pq = take(2 * g.nvox * sizeof(double));
  L.phase = take(g.nvox);
  L.params = take(256 * sizeof(PhaseC));
  L.aniso = take(aniso_words(g) * sizeof(double));
  L.tw = take(size_t(g.n0 + g.n1 + g.n2) * 2 * w);
  L.partials = take(size_t(g.xblocks) * kNAvg * sizeof(double));
  L.ctl = take(sizeof(Ctl));
  L.tot = take(64 * sizeof(double));
  L.gtab = take(green_table_bytes(g, w));
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// Field read-back (mp_get_fields, mp_batch_get_fields, served requests)
// ---------------------------------------------------------------------------
// Where field f of a state lives: e, gamma in the FP64 strain buffer, t, m in
// the committed stresses (bulk type, w bytes), p, q in the FP64 p, q buffer.
struct FieldSrc {
  const unsigned char* p;
  long count;   // values
  bool f32;     // stored as float
};

inline FieldSrc field_source(const unsigned char* E, const unsigned char* out_tm, const unsigned char* out_pq,
                             long n, size_t w, int field) {
  switch (field) {
    case MP_FIELD_E: return {E, 9 * n, false};
    case MP_FIELD_GAMMA: return {E + 9 * n * sizeof(double), 9 * n, false};
    case MP_FIELD_T: return {out_tm, 9 * n, w == sizeof(float)};
    case MP_FIELD_M: return {out_tm + 9 * n * w, 9 * n, w == sizeof(float)};
    case MP_FIELD_P: return {out_pq, n, false};
    default: return {out_pq + n * sizeof(double), n, false};
  }
}

constexpr uint32_t kFieldMask = (1u << 6) - 1;

inline mp_status check_field_args(uint32_t mask, void* const* dst) {
  if (mask & ~kFieldMask) return fail(MP_E_INVALID, "field mask has bits beyond MP_FIELD_Q");
  if (!mask) return MP_OK;
  if (!dst) return fail(MP_E_INVALID, "dst is NULL");
  for (int f = 0; f < 6; ++f)
    if ((mask >> f) & 1u && !dst[f]) return fail(MP_E_INVALID, "dst[" + std::to_string(f) + "] is NULL");
  return MP_OK;
}

// Copy the fields of `mask` into dst[field] as FP64 values.  Device
// destinations: enqueued on s (a float source is widened by k_widen), no
// wait; host destinations: the call waits for the copies.
inline mp_status copy_fields(const unsigned char* E, const unsigned char* out_tm, const unsigned char* out_pq,
                             long n, size_t w, uint32_t mask, void* const* dst, int dst_is_device,
                             hipStream_t s) {
  mp_status st = check_field_args(mask, dst);
  if (st != MP_OK || !mask) return st;
  std::vector<float> tmp;
  for (int f = 0; f < 6; ++f) {
    if (!((mask >> f) & 1u)) continue;
    const FieldSrc src = field_source(E, out_tm, out_pq, n, w, f);
    double* out = static_cast<double*>(dst[f]);
    if (dst_is_device) {
      if (src.f32) {
        hipLaunchKernelGGL(k_widen<float>, dim3(unsigned((src.count + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const float*>(src.p), out, src.count);
        HIP_TRY(hipGetLastError());
      } else {
        HIP_TRY(hipMemcpyAsync(out, src.p, src.count * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
    } else if (src.f32) {
      tmp.resize(src.count);
      HIP_TRY(hipMemcpyAsync(tmp.data(), src.p, src.count * sizeof(float), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (long i = 0; i < src.count; ++i) out[i] = double(tmp[i]);
    } else {
      HIP_TRY(hipMemcpyAsync(out, src.p, src.count * sizeof(double), hipMemcpyDeviceToHost, s));
    }
  }
  if (!dst_is_device) HIP_TRY(hipStreamSynchronize(s));
  return MP_OK;
}

inline PhaseC derive(const mp_phase& c) {
  PhaseC d{};
  d.t.lam = c.lambda; d.t.mu = c.mu; d.t.kap = c.kappa;
  d.t.tY = c.tY; d.t.tH = c.tH; d.t.a1 = c.a1;
  d.t.a2 = c.a1 * c.mu / c.kappa;
  d.t.aid = -1.0;
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


// Isotropic reference medium (Alg. 2: A0 = <A>, B0 = <B>): the unweighted
// mean of each modulus over the phases present (default), the volume average,
// or given.  With MP_REF_TENSOR_* the matching mean of the constants is kept
// beside the tensors (the kernels then use the tensors).
inline mp_status reference_medium(const mp_problem* prob, long nvox, RefC* out) {
  double refv[6] = {0, 0, 0, 0, 0, 0};
  if (prob->ref_mode == MP_REF_EXPLICIT) {
    const mp_phase& r = prob->ref;
    const double v[6] = {r.lambda, r.mu, r.kappa, r.alpha, r.beta, r.gamma};
    std::memcpy(refv, v, sizeof v);
  } else if (prob->ref_mode == MP_REF_GEOMETRIC_MEAN) {
    std::vector<long> count(prob->n_phases, 0);
    for (long i = 0; i < nvox; ++i) count[prob->phase[i]]++;
    double prod[6] = {1, 1, 1, 1, 1, 1};
    int present = 0;
    for (int i = 0; i < prob->n_phases; ++i) {
      if (!count[i]) continue;
      const mp_phase& c = prob->phases[i];
      const double v[6] = {c.lambda, c.mu, c.kappa, c.alpha, c.beta, c.gamma};
      for (int k = 0; k < 6; ++k) prod[k] *= v[k];
      ++present;
    }
    for (int k = 0; k < 6; ++k) refv[k] = std::pow(prod[k], 1.0 / present);
  } else {
    std::vector<long> count(prob->n_phases, 0);
    for (long i = 0; i < nvox; ++i) count[prob->phase[i]]++;
    double wsum = 0;
    for (int i = 0; i < prob->n_phases; ++i) {
      if (!count[i]) continue;
      const bool by_phase = prob->ref_mode == MP_REF_PHASE_MEAN || prob->ref_mode == MP_REF_TENSOR_PHASE_MEAN;
      const double wgt = by_phase ? 1.0 : double(count[i]);
      const mp_phase& c = prob->phases[i];
      const double v[6] = {c.lambda, c.mu, c.kappa, c.alpha, c.beta, c.gamma};
      for (int k = 0; k < 6; ++k) refv[k] += wgt * v[k];
      wsum += wgt;
    }
    for (int k = 0; k < 6; ++k) refv[k] /= wsum;
  }
  const RefC r{refv[0], refv[1], refv[2], refv[3], refv[4], refv[5]};
  if (!(r.lam + 2 * r.mu > 0) || !(r.mu > 0) || !(r.kap > 0) || !(r.gam > 0) ||
      !(r.alp + r.bet + r.gam > 0))
    return fail(MP_E_INVALID, "reference medium is not positive definite");
  *out = r;
  return MP_OK;
}

// Coefficients of the real symmetric Fourier symbol S(xi) of a general
// reference medium (the form green_apply_gen factors): entry e of the upper
// triangle, row by row, is sum_m G[10 e + m] mono_m(xi) with the monomials
// xi1^2, xi2^2, xi3^2, xi1 xi2, xi1 xi3, xi2 xi3, xi1, xi2, xi3, 1.
//   S_uu[l][j]   = A0_alkj xi_a xi_k
//   S_upsi[l][j] = xi_a C_alj,            C_abj = A0_abkl eps_lkj
//   S_psipsi[l][j] = B0_lkjn xi_k xi_n - F_lj,  F_lj = eps_lkm C_kmj
inline void green_symbol(const mp_aniso& r, double* G) {
  auto eps = [](int i, int j, int k) {
    return double((i - j) * (j - k) * (k - i)) / 2.0;   // Levi-Civita on 0..2
  };
  auto quad = [](int a, int k) { return a == k ? a : (a + k == 1 ? 3 : (a + k == 2 ? 4 : 5)); };
  auto A = [&](int k, int l, int m, int n) { return r.A[27 * k + 9 * l + 3 * m + n]; };
  auto B = [&](int l, int k, int m, int n) { return r.B[27 * l + 9 * k + 3 * m + n]; };
  double C[3][3][3] = {}, F[3][3] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) C[a][b][j] += A(a, b, k, l) * eps(l, k, j);
  for (int l = 0; l < 3; ++l)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) F[l][j] += eps(l, k, m) * C[k][m][j];
  std::fill(G, G + kSymEntries * kSymCoef, 0.0);
  for (int i = 0, e = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j, ++e) {
      double* g = G + kSymCoef * e;
      if (j < 3) {          // u-u
        for (int a = 0; a < 3; ++a)
          for (int k = 0; k < 3; ++k) g[quad(a, k)] += A(a, i, k, j);
      } else if (i < 3) {   // u-psi
        for (int a = 0; a < 3; ++a) g[6 + a] += C[a][i][j - 3];
      } else {              // psi-psi
        for (int k = 0; k < 3; ++k)
          for (int n = 0; n < 3; ++n) g[quad(k, n)] += B(i - 3, k, j - 3, n);
        g[9] -= F[i - 3][j - 3];
      }
    }
}

}  // namespace mp
