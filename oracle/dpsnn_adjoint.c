/*
 * dpsnn_adjoint.c -- FP64 oracle of the surrogate-gradient adjoint (backpropagation through
 * time) of the simulation step, and of a smooth "soft" version of the step used to check
 * the adjoint by finite differences.
 *
 * TEST INFRASTRUCTURE ONLY (see dpsnn_oracle.h).  The paper itself has no gradients; the
 * method differentiated here is its time-driven LIF + calcium-AHP step with delayed
 * synapses (sections 1 and 2), with the spike's derivative replaced by a surrogate.
 *
 * Forward quantities of neuron j at step u: V(u-1), Ca(u-1) (state before the step), the
 * pre-threshold potential V~(u), the spike s(u) and the refractory flag r(u).  The step is
 *     V~(u) = P_m V(u-1) - gamma Ca(u-1) + I(u),   I(u) = sum of w over synapses delivered
 *     V(u)  = V~(u) (1 - s(u)) + V_reset s(u)
 *     Ca(u) = P_c Ca(u-1) + alpha s(u)
 * (refractory steps hold V at V_reset and pass no gradient).  With nu(u) = dL/dV~(u),
 * lambda(u) = dL/dV(u), mu(u) = dL/dCa(u) and e(u) = dL/ds(u), the reverse recursion for
 * u = T-1 .. 0 is
 *     e(u)  = dL/ds(u)|direct + sum_{k in row(j)} w_k nu_{tgt k}(u + d_k)
 *             + lambda(u) (V_reset - V~(u)) + alpha mu(u)
 *     nu(u) = (1 - r(u)) [ lambda(u) (1 - s(u)) + e(u) sigma'(V~(u) - theta) ]
 *     lambda(u-1) = P_m nu(u),   mu(u-1) = -gamma nu(u) + P_c mu(u)
 * with nu beyond T zero, and the parameter gradients
 *     dL/dw_k   = sum_u s_pre(u) nu_{tgt k}(u + d_k)
 *     dL/dP_m   = sum_{j,u} V(u-1) nu(u),     dL/dgamma = - sum_{j,u} Ca(u-1) nu(u).
 * sigma' is the fast-sigmoid surrogate 1 / (1 + beta |x|)^2.  The same code is the exact
 * gradient of the soft model, whose spike is S(x) = 1/beta + x / (1 + beta |x|) (so that
 * S' = sigma'), with no refractory period.
 *
 * A loss may also depend on V~ directly: dl_dvt (nullable) adds dL/dV~(u)|direct inside the
 * bracket of nu.  With sigma' = 0 (beta -> infinity) and the spikes and refractory flags
 * held fixed, the recursion is then the exact gradient of the step with a frozen spike mask
 * (refractory steps hold V at V_reset, reset where s = 1), which finite differences check.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "dpsnn_oracle.h"

static double surrogate(double x, double beta) {
  double a = 1.0 + beta * fabs(x);
  return 1.0 / (a * a);
}

int orc_adjoint(const orc_adj_params_t* k, int64_t n, int64_t T, const int64_t* row_ptr,
                const int32_t* tgt, const uint8_t* dly, const double* w, const double* v_prev,
                const double* ca_prev, const double* v_tilde, const double* s, const uint8_t* r,
                const double* dl_ds, const double* dl_dvt, double* grad_w, double* grad_pm,
                double* grad_gamma) {
  int32_t dmax = 0;
  for (int64_t e = 0; e < row_ptr[n]; ++e)
    if (dly[e] > dmax) dmax = dly[e];
  /* nu of all steps, [T][n]; steps >= T are zero */
  double* nu = (double*)calloc((size_t)T * (size_t)n, sizeof(double));
  double* lam = (double*)calloc((size_t)n, sizeof(double));
  double* mu = (double*)calloc((size_t)n, sizeof(double));
  if (!nu || !lam || !mu) { free(nu); free(lam); free(mu); return -1; }
  memset(grad_w, 0, sizeof(double) * (size_t)row_ptr[n]);
  double gpm = 0.0, ggam = 0.0;
  for (int64_t u = T - 1; u >= 0; --u) {
    for (int64_t j = 0; j < n; ++j) {
      size_t o = (size_t)u * (size_t)n + (size_t)j;
      /* recurrent term: future adjoints of the targets of j's synapses */
      double gsum = 0.0;
      for (int64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
        int64_t t = u + dly[e];
        if (t < T) gsum += w[e] * nu[(size_t)t * (size_t)n + (size_t)tgt[e]];
      }
      double ej = dl_ds[o] + gsum + lam[j] * (k->vreset - v_tilde[o]) + k->alpha * mu[j];
      double nuj = 0.0;
      if (!r[o]) {
        nuj = lam[j] * (1.0 - s[o]) + ej * surrogate(v_tilde[o] - k->theta, k->beta);
        if (dl_dvt) nuj = nuj + dl_dvt[o];
      }
      nu[o] = nuj;
      gpm += v_prev[o] * nuj;
      ggam += -ca_prev[o] * nuj;
      lam[j] = k->pm * nuj;
      mu[j] = -k->gamma * nuj + k->pc * mu[j];
    }
  }
  /* weight gradients: every delivery of a (possibly soft) spike */
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      double acc = 0.0;
      for (int64_t u = 0; u + dly[e] < T; ++u) {
        double si = s[(size_t)u * (size_t)n + (size_t)i];
        if (si != 0.0) acc += si * nu[(size_t)(u + dly[e]) * (size_t)n + (size_t)tgt[e]];
      }
      grad_w[e] = acc;
    }
  }
  *grad_pm = gpm;
  *grad_gamma = ggam;
  free(nu); free(lam); free(mu);
  return 0;
}

/* Soft model forward in FP64: same step with the spike S(V~ - theta), soft reset and soft
 * delivery, no refractory period.  External input: the same Poisson counts as the hard
 * model (word j mod 4 of Philox at counter (j / 4, u, 0, EXT)), times J_ext.  Outputs are
 * [T][n]. */
int orc_soft_forward(const orc_config_t* cfg, const orc_adj_params_t* k, int64_t n, int64_t T,
                     const int64_t* row_ptr, const int32_t* tgt, const uint8_t* dly,
                     const double* w, double* v_prev, double* ca_prev, double* v_tilde,
                     double* s) {
  int32_t dmax = 0;
  for (int64_t e = 0; e < row_ptr[n]; ++e)
    if (dly[e] > dmax) dmax = dly[e];
  int64_t D = dmax + 1;
  double* ring = (double*)calloc((size_t)D * (size_t)n, sizeof(double));
  double* v = (double*)malloc(sizeof(double) * (size_t)n);
  double* ca = (double*)calloc((size_t)n, sizeof(double));
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!ring || !v || !ca || !next) { free(ring); free(v); free(ca); free(next); return -1; }
  double jext = rint(cfg->j_ext * 65536.0) / 65536.0;
  for (int64_t j = 0; j < n; ++j) v[j] = (double)orc_initial_v(cfg, j);
  for (int64_t u = 0; u < T; ++u) {
    orc_ext_counts(cfg, u, 0, n, next);
    double* in = ring + (u % D) * n;
    for (int64_t j = 0; j < n; ++j) {
      size_t o = (size_t)u * (size_t)n + (size_t)j;
      double cur = in[j] + (double)next[j] * jext;
      in[j] = 0.0;
      double vt = k->pm * v[j] - k->gamma * ca[j] + cur;
      double x = vt - k->theta;
      double sj = 1.0 / k->beta + x / (1.0 + k->beta * fabs(x));
      v_prev[o] = v[j];
      ca_prev[o] = ca[j];
      v_tilde[o] = vt;
      s[o] = sj;
      v[j] = vt * (1.0 - sj) + k->vreset * sj;
      ca[j] = k->pc * ca[j] + k->alpha * sj;
    }
    for (int64_t i = 0; i < n; ++i) {
      double si = s[(size_t)u * (size_t)n + (size_t)i];
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        ring[((u + dly[e]) % D) * n + tgt[e]] += w[e] * si;
    }
  }
  free(ring); free(v); free(ca); free(next);
  return 0;
}
