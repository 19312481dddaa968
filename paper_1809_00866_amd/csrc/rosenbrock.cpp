// Rosenbrock (linearly implicit Runge-Kutta) time step (Sec. 2.2, Alg. ros):
// one FGMRES solve per stage with the Jacobian of the step's initial state,
// stage right-hand sides built from the residual at the stage state and the
// earlier stage increments.  Every vector operation runs on the device.
#include <algorithm>
#include <cmath>

#include "context.h"

using namespace dgc;

extern "C" {

dg_status dg_rosenbrock_step(dg_context* c, const double* w, double dt, const dg_rosenbrock* k,
                             const dg_solve_opts* opts, double* w_next, dg_solve_stats* stats, void* stream) {
  if (!c || !w || !k || !opts || !w_next) return fail(DG_ERR_ARG, "null argument");
  if (w == w_next) return fail(DG_ERR_ARG, "w and w_next may not alias");
  if (k->n_stages < 1 || k->n_stages > DG_ROS_MAX_STAGES) return fail(DG_ERR_ARG, "n_stages must lie in 1..6");
  if (!(dt > 0.0) || !(k->gamma > 0.0) || !std::isfinite(dt) || !std::isfinite(k->gamma))
    return fail(DG_ERR_ARG, "dt and gamma must be positive and finite");
  hipStream_t s = (hipStream_t)stream;
  const int ns = k->n_stages;
  const int64_t n = c->ndof;
  const int64_t need = (int64_t)(ns + 2) * n;
  dg_status st;
  if (c->ros_len < need) {
    dfree(c->d_ros);
    c->d_ros = nullptr;
    c->ros_len = 0;
    if ((st = dalloc(&c->d_ros, (size_t)need)) != DG_OK) return st;
    c->ros_len = need;
  }
  double* dw = c->d_ros;                  // stage increments dw_0 .. dw_{ns-1}
  double* ws = c->d_ros + (size_t)ns * n;  // stage state w + dp
  double* rhs = ws + n;
  const double shift = 1.0 / (k->gamma * dt);
  dg_solve_stats tot{};
  tot.converged = 1;
  for (int si = 0; si < ns; ++si) {
    double* dws = dw + (size_t)si * n;
    // ws = w + sum a[si][o] dw_o ; rhs = -R(ws) - (1/dt) sum c[si][o] dw_o
    HIPCHK(dgk::launch_axpby(n, 1.0, w, 0.0, w, ws, s));
    for (int o = 0; o < si; ++o)
      if (k->a[si][o] != 0.0) HIPCHK(dgk::launch_axpby(n, 1.0, ws, k->a[si][o], dw + (size_t)o * n, ws, s));
    if ((st = eval_residual(c, false, ws, nullptr, 0.0, rhs, s)) != DG_OK) return st;
    HIPCHK(dgk::launch_axpby(n, -1.0, rhs, 0.0, rhs, rhs, s));
    // (the mass form: only the variables with a time derivative)
    for (int o = 0; o < si; ++o)
      if (k->c[si][o] != 0.0)
        HIPCHK(dgk::launch_axpby(c->mass_len, 1.0, rhs, -k->c[si][o] / dt, dw + (size_t)o * n, rhs, s));
    HIPCHK(dgk::launch_fill(dws, n, 0.0, s));
    dg_solve_stats sst{};
    st = dg_fgmres_solve(c, w, shift, rhs, dws, opts, &sst, stream);
    if (st != DG_OK && st != DG_NOT_CONVERGED) return st;
    tot.iters += sst.iters;
    tot.restarts += sst.restarts;
    tot.converged = tot.converged && sst.converged;
    tot.rel_res_est = std::max(tot.rel_res_est, sst.rel_res_est);
    tot.rel_res_true = std::max(tot.rel_res_true, sst.rel_res_true);
    tot.rho = std::max(tot.rho, sst.rho);
    tot.ms_solve += sst.ms_solve;
    tot.fallbacks += sst.fallbacks;
    tot.ms_setup = sst.ms_setup;
  }
  HIPCHK(dgk::launch_axpby(n, 1.0, w, 0.0, w, w_next, s));
  for (int si = 0; si < ns; ++si)
    if (k->m[si] != 0.0) HIPCHK(dgk::launch_axpby(n, 1.0, w_next, k->m[si], dw + (size_t)si * n, w_next, s));
  if (stats) *stats = tot;
  return tot.converged ? DG_OK : DG_NOT_CONVERGED;
}

}  // extern "C"
