// The per-check decisions of one PDHG run: KKT quantities from the FP64
// check scalars, the eps_rel milestone, termination, the FP32 -> FP64
// hand-over, the adaptive restart and the primal-weight update.  One
// function serves the device (the engine's check kernel, one thread per
// resident instance) and the host (scenario batches, one call per lane).
// Internal; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/uc_lp.h"
#include "uclp_dev.h"

namespace uclp {

// Options that enter the decisions (copied from uc_lp_opts) and the data
// norms of the instance.
struct ChkParams {
  int32_t mode;  // uc_lp_precision of the solve
  int32_t K;     // iterations per check interval
  int32_t restart_to_current;
  int32_t fp32_stall_checks;
  int64_t iter_limit;
  double eps_rel, eps_polish, eps_gap_rel, eps_abs_feas;
  double eps_refine;  // UC_LP_FP32_REFINE: target of each correction problem
  double restart_sufficient, restart_necessary, restart_artificial;
  double pw_smoothing, pw_max_change, pw_integral, pw_balance;
  double norm_b, norm_c, obj_offset;
  // > 0: denominator of the relative gap in place of 1 + |pobj| + |dobj|
  // (a correction problem measures its gap on the scale of the refined point)
  double gap_den;
  // UC_LP_FP32_REFINE, correction problems: the balance gain, and the factor
  // over the round's best error at which a round ends (0: never)
  double pw_balance_inner, inner_diverge;
};

// State of one run between checks, and what the last check found.
struct ChkState {
  int32_t prec;       // 1: FP32 phase, 0: FP64 phase
  int32_t status;     // UC_LP_RUNNING, or the terminal status of the run
  int32_t promote;    // the last check ended the FP32 phase
  int32_t restart;    // the last check's restart flag for the finish kernel (0, 1, 2)
  int32_t r_start_set, r_prev_set, gap_phase, eps_reached;
  int32_t round;      // UC_LP_FP32_REFINE: 0 the base solve, k > 0 correction problem k
  int32_t pad_;
  double eta, omega;
  int64_t k_inner;      // steps since the last restart
  int64_t phase_total;  // steps in the current precision phase
  int64_t iters, iters64, restarts, checks, best_check;
  double r_start, r_prev, pw_int, best_kkt;
  // the last check
  double pobj, dobj, rel_primal, rel_dual, rel_gap, rel_kkt, abs_primal_inf, fp_residual;
  // the eps_rel milestone
  int64_t iters_at_eps;
  double pobj_at_eps, rel_kkt_at_eps, rel_gap_at_eps;
  uint64_t tick_at_eps;  // device clock at the milestone (0 from the host)
};

// One check of a run from the reduced FP64 scalars q (see RowQ / ColQ).
// `stop` (0 = none) is a terminal status the caller imposes (time limit,
// cancel); `tick` stamps the milestone.  Updates st; the caller reads
// st.status, st.promote and st.restart.
__host__ __device__ inline void check_step(ChkState& st, const ChkParams& p, const double* q, int32_t stop,
                                           uint64_t tick) {
  const int K = p.K;
  // KKT quantities (unscaled, original problem)
  const double rho_p = sqrt(fmax(q[RQ_RES2], 0.0));
  const double rho_d = sqrt(fmax(q[RQ_N + CQ_DRES2] + q[RQ_YNEG2], 0.0));
  // a lower bound ylo on the inequality duals adds -ylo'(A_G x - b_G) to
  // the primal objective (RQ_YLOR; zero unless ylo is in use)
  const double pobj = q[RQ_N + CQ_CX] - q[RQ_YLOR] + p.obj_offset;
  const double dobj = q[RQ_BY] + q[RQ_N + CQ_LBUB] + p.obj_offset;
  st.pobj = pobj;
  st.dobj = dobj;
  st.rel_primal = rho_p / (1.0 + p.norm_b);
  st.rel_dual = rho_d / (1.0 + p.norm_c);
  st.rel_gap = fabs(pobj - dobj) / (p.gap_den > 0 ? p.gap_den : 1.0 + fabs(pobj) + fabs(dobj));
  st.rel_kkt = fmax(st.rel_primal, fmax(st.rel_dual, st.rel_gap));
  st.abs_primal_inf = q[RQ_RESMAX];
  st.iters += K;
  if (st.prec == 0) st.iters64 += K;
  st.phase_total += K;
  st.promote = 0;
  st.restart = 0;
  const int64_t k_end = st.k_inner + K;
  // ||z - T(z)||_P in the metric of the PDHG step, P = [[I/tau, A'], [A, I/sigma]]
  const double dx2 = q[RQ_N + CQ_DX2], dy2 = q[RQ_DY2], cross = q[RQ_DYADX];
  const double rfp = sqrt(fmax(st.omega / st.eta * dx2 + dy2 / (st.omega * st.eta) + 2.0 * cross, 0.0));
  st.fp_residual = rfp;
  // a correction problem of iterative refinement: its own target; the
  // absolute feasibility test applies to the refined point (host side)
  const bool refine_mode = p.mode == UC_LP_FP32_REFINE;
  const bool inner = refine_mode && st.round > 0;
  const bool feas_ok = inner || p.eps_abs_feas <= 0 || st.abs_primal_inf <= p.eps_abs_feas;
  const bool finite = isfinite(st.rel_kkt) && isfinite(rfp) && isfinite(pobj);
  bool terminate = false, promote = false;
  int32_t status = UC_LP_RUNNING;
  if (!finite) {
    terminate = true;
    status = UC_LP_NUMERICAL;
  } else {
    if (!st.eps_reached && !inner && st.rel_kkt <= p.eps_rel && feas_ok) {
      st.eps_reached = 1;
      st.pobj_at_eps = pobj;
      st.rel_kkt_at_eps = st.rel_kkt;
      st.rel_gap_at_eps = st.rel_gap;
      st.iters_at_eps = st.iters;
      st.tick_at_eps = tick;
    }
    const bool polish_mode = p.mode == UC_LP_FP32_MIXED_POLISH;
    const bool polish_phase = polish_mode && st.prec == 0;
    const double target = polish_phase ? p.eps_polish : inner ? p.eps_refine : p.eps_rel;
    // outside the polish and refinement modes a returned point may also have
    // to close the gap
    const bool gap_rule = !polish_mode && !refine_mode && p.eps_gap_rel > 0;
    const bool gap_ok = !gap_rule || st.rel_gap <= p.eps_gap_rel;
    if (st.rel_kkt <= target && feas_ok) {
      // the FP32 phase ends: polish in FP64, or (refinement) the host folds
      // the point into the refined one and forms the next correction problem
      if ((polish_mode || refine_mode) && st.prec == 1) {
        promote = true;
      } else if (gap_ok) {
        terminate = true;
        status = UC_LP_OPTIMAL;
      }
    }
    // an FP32 phase that stopped improving continues in FP64.  Progress is
    // the KKT error, and past the eps_rel milestone under the gap rule the
    // larger of it and the gap, both relative to their targets
    ++st.checks;
    if (st.prec == 1 && !terminate && !promote) {
      const bool continuing = gap_rule && st.eps_reached;
      const double err = continuing ? fmax(st.rel_kkt, st.rel_gap * (target / p.eps_gap_rel)) : st.rel_kkt;
      if (continuing && !st.gap_phase) {
        st.gap_phase = 1;  // the progress measure changes: its window starts afresh
        st.best_check = 0;
      }
      if (st.best_check == 0 || err < 0.9 * st.best_kkt) {
        st.best_kkt = err;
        st.best_check = st.checks;
      } else if (inner && p.inner_diverge > 0 && err > p.inner_diverge * st.best_kkt) {
        // a correction problem moving away from the point it corrects
        // (a primal weight run away): the round ends before it undoes more
        promote = true;
      } else if (p.fp32_stall_checks > 0 &&
                 st.checks - st.best_check >= (inner ? 12 : 1) * (int64_t)p.fp32_stall_checks &&
                 (continuing || inner || st.best_kkt <= 10.0 * target)) {
        // a stall within a decade of the target (or of the gap past the
        // milestone) is taken for the FP32 floor.  A correction problem,
        // which is O(1)-scaled and far from that floor, gets twelve times
        // the window (restarted PDHG can take that long for 10% near 1e-8);
        // when it stalls, it ends its round wherever it stands
        promote = true;
      }
    }
    if (!terminate && st.iters >= p.iter_limit) {
      terminate = true;
      status = UC_LP_ITER_LIMIT;
    }
    if (!terminate && stop != 0) {
      terminate = true;
      status = stop;
    }
  }
  if (terminate) promote = false;
  if (!terminate && !promote) {
    if (!st.r_start_set) {
      st.r_start = rfp;
      st.r_start_set = 1;
    }
    bool rs = rfp <= p.restart_sufficient * st.r_start;
    if (!rs && rfp <= p.restart_necessary * st.r_start && st.r_prev_set && rfp > st.r_prev) rs = true;
    if (!rs && (double)k_end >= p.restart_artificial * (double)st.phase_total) rs = true;
    st.r_prev = rfp;
    st.r_prev_set = 1;
    if (rs) {
      const double dX = sqrt(fmax(q[RQ_N + CQ_DX0], 0.0));
      const double dY = sqrt(fmax(q[RQ_DY0], 0.0));
      if (dX > 1e-10 && dY > 1e-10) {
        // log w <- log w - th e - ki sum(e), e = log w - log(dY / dX)
        const double e = log(st.omega) - log(dY / dX);
        st.pw_int += e;
        double lw = log(st.omega) - p.pw_smoothing * e - p.pw_integral * st.pw_int;
        // residual balance: a primal residual above the dual one raises w
        const double gain = inner ? p.pw_balance_inner : p.pw_balance;
        if (gain > 0 && st.rel_primal > 0 && st.rel_dual > 0) lw += gain * log(st.rel_primal / st.rel_dual);
        double w = exp(lw);
        if (p.pw_max_change >= 1) w = fmin(fmax(w, st.omega / p.pw_max_change), st.omega * p.pw_max_change);
        st.omega = w;
      }
      st.k_inner = 0;
      st.r_start_set = 0;
      st.r_prev_set = 0;
      ++st.restarts;
      st.restart = p.restart_to_current ? 2 : 1;
    } else {
      st.k_inner = k_end;
    }
  }
  if (promote && !refine_mode) {
    // the FP64 phase starts at (x_hat, y_hat) as after a restart
    st.prec = 0;
    st.k_inner = 0;
    st.phase_total = 0;
    st.r_start_set = 0;
    st.r_prev_set = 0;
  }
  st.promote = promote ? 1 : 0;
  st.status = terminate ? status : UC_LP_RUNNING;
}

}  // namespace uclp
