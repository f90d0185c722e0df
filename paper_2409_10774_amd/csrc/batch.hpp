// Resident batches of RVEs: many independent cells of different sizes
// iterate together, each with its own load path, convergence and step
// control, all of it on the device.
//
// Every resident RVE has a descriptor (Rve) in device memory holding its
// x-pass and axis-pass arguments, its loop control block and its place in
// its load path.  One loop iteration of the whole batch is, per shape class,
// a y-forward, z (forward + Green + inverse), y-inverse and x pass, then one
// row reduction and one control kernel for all classes.  The kernels run a
// persistent grid over work lists that the control kernel rebuilds after
// every iteration, so RVEs that have converged drop out at once and the
// launch sequence never changes: it is captured once as a graph of several
// iterations and replayed.
//
// Per-RVE state machine (advanced only by k_batch_ctl):
//   TRANS  the next x pass commits the converged step (if commit) and opens
//          the next one (if init); spectral passes skip the RVE
//   RUN    a loop iteration of the current step
//   DONE   last step committed, or a step failed (max_iter: committed;
//          diverged: not committed); results are readable
// An admitted RVE starts in TRANS with init only.
#pragma once

#include "kernels.hpp"

namespace mp {

constexpr int kMaxSlots = 512;    // resident RVEs per batch
constexpr int kMaxClasses = 8;    // shape classes per batch
constexpr int kRec = 48;          // doubles per step record

enum RvState { RV_EMPTY = 0, RV_RUN = 1, RV_TRANS = 2, RV_DONE = 3 };
enum RvStatus { RVS_OK = 0, RVS_NOT_CONVERGED = 1, RVS_DIVERGED = 2 };

template <class T>
struct Rve {
  XArgs<T> x;
  AxisArgs<T> y, z;
  Ctl ctl;
  const double* times;   // n_steps + 1: times[0] start state, step s ends at times[s + 1]
  const double* Ep;      // [n_steps][9] prescribed E
  const double* Gp;      // [n_steps][9] prescribed Gamma
  double* rec;           // [n_steps][kRec]: 40 average sums, err, iters, 4 err parts, reserved
  double tot[kNAvg];     // reduced rows of the last x pass
  double pend[8];        // err, iters, err parts, reserved of the step awaiting commit
  double tol;
  long nvox;
  int xblocks;
  int state, cls, step, n_steps, committed, status;
  int fixed, max_iter, norm;
  long iters_total;
};

struct Lists {
  int ns[kMaxClasses];   // RVEs iterating this iteration (RUN): spectral + ITER x passes
  int nt[kMaxClasses];   // RVEs between steps (TRANS): TRANS x pass
  int active;            // RVEs in RUN or TRANS
  int launches;          // control-kernel passes (loop iterations of the batch)
  int st[kMaxSlots];     // state of every slot
  int s[kMaxClasses][kMaxSlots];
  int t[kMaxClasses][kMaxSlots];
};

// Work distribution: block b takes work items b, b + G, b + 2G, ... of its
// pass (G = grid size).  Every item of a pass costs the same, so a grid that
// is an integer multiple of what the chip holds at once loses nothing to
// imbalance; the grids are large (several times the chip's block slots), and
// in the common case a block takes a single item.  No atomics: a shared
// work counter serialises across the chip's L2 domains.
// x pass of one shape class: ITER over the RUN list, or TRANS over the
// TRANS list (commit of an RVE's step and first iterate of its next).  In
// low precision the ITER kernel also takes the TRANS items, after its own:
// the two lists hold different RVEs, each item runs its own pass body, and a
// class needs one x kernel per loop iteration instead of two (the 10 x 10
// length-scale sweep of 16^3 cells: 3.6 against 3.69 s).  The TRANS body
// then shares the ITER kernel's register budget, which in FP64 costs the
// loop body spills (a basic FP64 batch 2 % slower): FP64 keeps the TRANS
// kernel apart.  AN: the Eq. 5 variant of the pass body, for a class holding
// an RVE with Eq. 5 phases (an RVE without them takes the same arithmetic in
// either variant); AL (FP64 ITER only): each RVE runs the
// augmented-Lagrangian or the basic loop body by its own flag, for a class
// holding an augmented-Lagrangian RVE
template <class T>
constexpr bool x_merged() { return sizeof(T) < sizeof(double); }

template <class T, int MODE, int N0, bool AN, bool AL = false>
__global__ void __launch_bounds__((XShape<T, N0>::NTHR), (AL ? x_min_waves<T, MODE, true>() : x_min_waves<T, MODE>())) k_batch_x(const Rve<T>* __restrict__ rv,
                                                              const Lists* __restrict__ ls, int cls,
                                                              int tiles) {
  using X = XShape<T, N0>;
  __shared__ cx<T> lds[X::NPK * N0];
  __shared__ cx<T> lds2[X::NPK * N0];
  __shared__ double red[X::NTHR / 64][kRed];
  __shared__ cx<T> twl[N0];
  constexpr bool STASH = sizeof(T) < sizeof(double) && MODE == X_ITER;
  __shared__ double stash[STASH ? 9 * X::NTHR : 1];
  // this kernel's own items, then (low precision ITER) the TRANS items
  constexpr bool WITH_TRANS = MODE == X_ITER && x_merged<T>();
  const int n = MODE == X_ITER ? ls->ns[cls] : ls->nt[cls];
  const int* list = MODE == X_ITER ? ls->s[cls] : ls->t[cls];
  const int nt = WITH_TRANS ? ls->nt[cls] : 0;
  const long total = long(n) * tiles, total_t = long(nt) * tiles;   // (RVE, tile) items, two levels each
  if (total == 0 && total_t == 0) return;
  // item slots: the own items' x_grid, then the TRANS items' (x_grid is a
  // multiple of 16 for one level per block, so the level pairing of x_item
  // holds in both ranges)
  const long gi = x_grid<X::LPB>(total), gend = gi + x_grid<X::LPB>(total_t);
  // every RVE of a class has the same twiddles: load them once per block
  load_twiddles<T, N0, X::NTHR>(twl, glob(rv[n > 0 ? list[0] : ls->t[cls][0]].x.tw), threadIdx.x);
  // items w -> ((RVE, tile), first level) as x_item; the grid is a multiple
  // of 16, so the two levels of an item in separate blocks run on one XCD
  for (long w = blockIdx.x; w < gend; w += gridDim.x) {
    const bool trans = WITH_TRANS && w >= gi;
    long u;
    int lvl;
    x_item<X::LPB>(trans ? w - gi : w, &u, &lvl);
    if (u >= (trans ? total_t : total)) continue;
    const int slot = trans ? ls->t[cls][u / tiles] : list[u / tiles];
    const int tile = int(u % tiles);
    __syncthreads();   // the previous item is done with LDS
    if constexpr (WITH_TRANS) {
      if (trans) {
        xpass_tile<T, X_TRANS, N0, AN>(rv[slot].x, tile, lvl, tiles, lds, lds2, red, twl, fresh_tid(), false,
                                       false, stash);
        continue;
      }
    }
    if constexpr (AL && MODE == X_ITER && sizeof(T) == sizeof(double)) {
      // the scheme is uniform over the item (one RVE): the two bodies never
      // share one loop's registers
      if (rv[slot].x.al)
        xpass_tile<T, MODE, N0, AN, true>(rv[slot].x, tile, lvl, tiles, lds, lds2, red, twl, fresh_tid(),
                                          rv[slot].ctl.rd_incr, rv[slot].ctl.wr_incr, stash);
      else
        xpass_tile<T, MODE, N0, AN, false>(rv[slot].x, tile, lvl, tiles, lds, lds2, red, twl, fresh_tid(),
                                           rv[slot].ctl.rd_incr, rv[slot].ctl.wr_incr, stash);
    } else {
      xpass_tile<T, MODE, N0, AN>(rv[slot].x, tile, lvl, tiles, lds, lds2, red, twl, fresh_tid(),
                                  rv[slot].ctl.rd_incr, rv[slot].ctl.wr_incr, stash);
    }
  }
}

// y or z pass of one shape class over its RUN RVEs; tile t of an RVE is
// (bx, by) = (t mod gx, t / gx)
template <class T, int MODE, int L, int TX>
__global__ void __launch_bounds__((AShape<L, TX>::NTHR), (axis_min_waves<T, L, TX>()))
    k_batch_axis(const Rve<T>* __restrict__ rv, const Lists* __restrict__ ls, int cls, int gx, int gy) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  __shared__ cx<T> twl[L];
  const int tiles = gx * gy;
  const int total = ls->ns[cls] * tiles;
  // every RVE of a class has the same twiddles: load them once per block
  if (int(blockIdx.x) < total) {
    const int s0 = ls->s[cls][blockIdx.x / tiles];
    load_twiddles<T, L, AShape<L, TX>::NTHR>(
        twl, glob((MODE == Y_FWD || MODE == Y_INV) ? rv[s0].y.tw : rv[s0].z.tw), threadIdx.x);
  }
  // round r covers items [r G, r G + n_r); within a round the items are
  // handed out XCD-aware (xcd_tile)
  for (int r0 = 0; r0 < total; r0 += gridDim.x) {
    const int nr = min(int(gridDim.x), total - r0);
    if (int(blockIdx.x) >= nr) break;
    const int w = r0 + xcd_tile(blockIdx.x, nr);
    const int slot = ls->s[cls][w / tiles];
    const int t = w % tiles;
    __syncthreads();
    const AxisArgs<T>& a = (MODE == Y_FWD || MODE == Y_INV) ? rv[slot].y : rv[slot].z;
    axis_tile<T, MODE, L, TX>(a, t % gx, t / gx, lds, twl, fresh_tid());
  }
}

// Row reductions of every x pass of the iteration: the kNPart error rows of
// each RUN RVE, then the kNAvg step-average rows of each committing TRANS RVE
// (same code and order as the single-RVE path).
template <class T>
__global__ void __launch_bounds__(256) k_batch_rows(Rve<T>* __restrict__ rv,
                                                    const Lists* __restrict__ ls, int ncls) {
  __shared__ double red[4];
  int total = 0;
  for (int c = 0; c < ncls; ++c) total += ls->ns[c] * kNPart + ls->nt[c] * kNAvg;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int u = w, c = 0, slot = 0, j = 0;
    bool iter = true;
    for (;; ++c) {
      if (u < ls->ns[c] * kNPart) {
        slot = ls->s[c][u / kNPart];
        j = u % kNPart;
        break;
      }
      u -= ls->ns[c] * kNPart;
      if (u < ls->nt[c] * kNAvg) {
        slot = ls->t[c][u / kNAvg];
        j = u % kNAvg;
        iter = false;
        break;
      }
      u -= ls->nt[c] * kNAvg;
    }
    Rve<T>& R = rv[slot];
    if (!iter && !R.x.commit) continue;
    __syncthreads();
    const double v = row_reduce(glob(R.x.partials) + (long)j * R.xblocks, R.xblocks,
                                iter && err_row_is_max(j), red);
    if (threadIdx.x == 0) R.tot[j] = v;
  }
}

// Control: advance every RVE's state machine (update = 1), then rebuild the
// work lists in slot order.  One block of kMaxSlots threads, thread i owns
// slot i.
template <class T>
__global__ void __launch_bounds__(kMaxSlots) k_batch_ctl(Rve<T>* rv, Lists* ls, int ncls, int update) {
  const int i = threadIdx.x;
  Rve<T>& R = rv[i];
  int state = R.state;
  if (update && state == RV_RUN) {
    err_finalize(R.tot, R.nvox, &R.ctl, R.x.mac);
    R.iters_total += 1;
    const int d = R.ctl.done;
    if (d == 3) {
      // diverged: the step is not committed and the RVE takes no further steps
      R.status = RVS_DIVERGED;
      state = RV_DONE;
    } else if (d) {
      R.pend[0] = R.ctl.err;
      R.pend[1] = R.ctl.iters;
      for (int f = 0; f < 4; ++f) R.pend[2 + f] = R.ctl.err_parts[f];
      R.pend[6] = 0.0;
      const bool failed = d == 2;
      if (failed) R.status = RVS_NOT_CONVERGED;
      const int next = R.step + 1;
      const bool last = failed || next >= R.n_steps;
      R.x.commit = 1;
      R.x.init = last ? 0 : 1;
      R.x.first = 0;
      if (!last) {
        // Alg. 2 linear extrapolation ratio (t_n - t_{n-1}) / (t_{n-1} - t_{n-2})
        R.x.r = (R.times[next + 1] - R.times[next]) / (R.times[next] - R.times[next - 1]);
        for (int c = 0; c < 9; ++c) {
          R.x.mac[c] = R.Ep[next * 9 + c];
          R.x.mac[9 + c] = R.Gp[next * 9 + c];
        }
        R.step = next;
      }
      state = RV_TRANS;
    }
  } else if (update && state == RV_TRANS) {
    if (R.x.commit) {
      double* rec = R.rec + (long)R.committed * kRec;
      for (int j = 0; j < kNAvg; ++j) rec[j] = R.tot[j];
      for (int j = 0; j < 7; ++j) rec[kNAvg + j] = R.pend[j];
      R.committed += 1;
    }
    if (R.x.init) {
      ctl_reset(&R.ctl, R.fixed, R.max_iter, R.tol, R.norm);
      state = RV_RUN;
    } else {
      state = RV_DONE;
    }
  }
  if (update) R.state = state;
  ls->st[i] = state;
  // work lists in slot order: a wave ballot per class, then the waves' counts
  // in order (prefix compaction)
  __shared__ int wcnt[2][kMaxSlots / 64];
  const int lane = i & 63, wv = i >> 6;
  const int cls = R.cls;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int c = 0; c < ncls; ++c) {
    const bool fs = cls == c && state == RV_RUN;
    const bool ft = cls == c && state == RV_TRANS;
    const unsigned long long bs = __ballot(fs), bt = __ballot(ft);
    if (lane == 0) {
      wcnt[0][wv] = __popcll(bs);
      wcnt[1][wv] = __popcll(bt);
    }
    __syncthreads();
    int os = 0, ot = 0;
    for (int w = 0; w < wv; ++w) {
      os += wcnt[0][w];
      ot += wcnt[1][w];
    }
    if (fs) ls->s[c][os + __popcll(bs & below)] = i;
    if (ft) ls->t[c][ot + __popcll(bt & below)] = i;
    if (i == kMaxSlots - 1) {
      ls->ns[c] = os + __popcll(bs);
      ls->nt[c] = ot + __popcll(bt);
    }
    __syncthreads();
  }
  const int active = __syncthreads_count(state == RV_RUN || state == RV_TRANS);
  if (i == 0) {
    ls->active = active;
    if (update) ls->launches += 1;
  }
}

}  // namespace mp
