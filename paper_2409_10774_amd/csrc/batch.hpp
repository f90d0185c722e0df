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
//   DONE   last step committed (or failed); results are readable
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
  double* rec;           // [n_steps][kRec]: 40 average sums, err, iters, 4 err parts, floor flag
  double tot[kNAvg];     // reduced rows of the last x pass
  double pend[8];        // err, iters, err parts, floor flag of the step awaiting commit
  double tol;
  long nvox;
  int xblocks;
  int state, cls, step, n_steps, committed, status;
  int fixed, max_iter, norm, window;
  long iters_total;
};

struct Lists {
  int nx[kMaxClasses];   // RVEs with an x pass this iteration (RUN or TRANS)
  int ns[kMaxClasses];   // RVEs with spectral passes this iteration (RUN)
  int active;            // RVEs in RUN or TRANS
  int launches;          // control-kernel passes (loop iterations of the batch)
  int st[kMaxSlots];     // state of every slot
  int x[kMaxClasses][kMaxSlots];
  int s[kMaxClasses][kMaxSlots];
};

// x pass of one shape class: ITER for RUN RVEs, TRANS for TRANS RVEs
template <class T, int N0>
__global__ void __launch_bounds__(XShape<N0>::NTHR) k_batch_x(const Rve<T>* rv, const Lists* ls,
                                                              int cls, int tiles) {
  using X = XShape<N0>;
  __shared__ cx<T> lds[X::NPK * N0];
  __shared__ double red[X::NTHR / 64][kRed];
  const long total = long(ls->nx[cls]) * tiles;
  for (long w = blockIdx.x; w < total; w += gridDim.x) {
    const int slot = ls->x[cls][w / tiles];
    const long tile = w % tiles;
    const Rve<T>& R = rv[slot];
    __syncthreads();   // the previous tile is done with LDS
    if (R.state == RV_RUN)
      xpass_tile<T, X_ITER, N0>(R.x, tile, tiles, lds, red);
    else
      xpass_tile<T, X_TRANS, N0>(R.x, tile, tiles, lds, red);
  }
}

// y or z pass of one shape class over its RUN RVEs; tile t of an RVE is
// (bx, by) = (t mod gx, t / gx)
template <class T, int MODE, int L, int TX>
__global__ void __launch_bounds__((AShape<L, TX>::NTHR)) k_batch_axis(const Rve<T>* rv, const Lists* ls,
                                                                      int cls, int gx, int gy) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tiles = gx * gy;
  const long total = long(ls->ns[cls]) * tiles;
  for (long w = blockIdx.x; w < total; w += gridDim.x) {
    const int slot = ls->s[cls][w / tiles];
    const int t = int(w % tiles);
    __syncthreads();
    const AxisArgs<T>& a = (MODE == Y_FWD || MODE == Y_INV) ? rv[slot].y : rv[slot].z;
    axis_tile<T, MODE, L, TX>(a, t % gx, t / gx, lds, threadIdx.x);
  }
}

// Row reductions of every x pass of the iteration: error rows of RUN RVEs,
// step-average rows of committing TRANS RVEs (same code and order as the
// single-RVE path).
template <class T>
__global__ void __launch_bounds__(256) k_batch_rows(Rve<T>* rv, const Lists* ls, int ncls) {
  __shared__ double red[4];
  long total = 0;
  for (int c = 0; c < ncls; ++c) total += long(ls->nx[c]) * kNAvg;
  for (long w = blockIdx.x; w < total; w += gridDim.x) {
    long u = w;
    int c = 0;
    while (u >= long(ls->nx[c]) * kNAvg) {
      u -= long(ls->nx[c]) * kNAvg;
      ++c;
    }
    const int slot = ls->x[c][u / kNAvg], j = int(u % kNAvg);
    Rve<T>& R = rv[slot];
    const bool iter = R.state == RV_RUN;
    if (iter ? j >= kNPart : !R.x.commit) continue;
    __syncthreads();
    const double v = row_reduce(R.x.partials + (long)j * R.xblocks, R.xblocks,
                                iter && err_row_is_max(j), red);
    if (threadIdx.x == 0) R.tot[j] = v;
  }
}

// Control: advance every RVE's state machine (update = 1), then rebuild the
// work lists in slot order.  One block of kMaxSlots threads, thread i owns
// slot i.
template <class T>
__global__ void __launch_bounds__(kMaxSlots) k_batch_ctl(Rve<T>* rv, Lists* ls, int ncls, int update) {
  __shared__ int st[kMaxSlots], cl[kMaxSlots];
  const int i = threadIdx.x;
  Rve<T>& R = rv[i];
  int state = R.state;
  if (update && state == RV_RUN) {
    err_finalize(R.tot, R.nvox, &R.ctl, R.x.mac);
    R.iters_total += 1;
    const int d = R.ctl.done;
    if (d) {
      R.pend[0] = R.ctl.err;
      R.pend[1] = R.ctl.iters;
      for (int f = 0; f < 4; ++f) R.pend[2 + f] = R.ctl.err_parts[f];
      R.pend[6] = d == 4 ? 1.0 : 0.0;
      const bool failed = d == 2 || d == 3;
      if (failed) R.status = d == 2 ? RVS_NOT_CONVERGED : RVS_DIVERGED;
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
      ctl_reset(&R.ctl, R.fixed, R.max_iter, R.tol, R.norm, R.window);
      state = RV_RUN;
    } else {
      state = RV_DONE;
    }
  }
  if (update) R.state = state;
  st[i] = state;
  cl[i] = R.cls;
  ls->st[i] = state;
  __syncthreads();
  if (i < ncls) {
    int nx = 0, ns = 0;
    for (int k = 0; k < kMaxSlots; ++k) {
      if (cl[k] != i) continue;
      if (st[k] == RV_RUN) {
        ls->s[i][ns++] = k;
        ls->x[i][nx++] = k;
      } else if (st[k] == RV_TRANS) {
        ls->x[i][nx++] = k;
      }
    }
    ls->nx[i] = nx;
    ls->ns[i] = ns;
  }
  if (i == kMaxSlots - 1) {
    int a = 0;
    for (int k = 0; k < kMaxSlots; ++k) a += (st[k] == RV_RUN || st[k] == RV_TRANS);
    ls->active = a;
    if (update) ls->launches += 1;
  }
}

}  // namespace mp
