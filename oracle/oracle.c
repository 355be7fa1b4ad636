/* FP64 CPU oracle for one Bayesian-optimization surrogate step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the GPU library.  Plain loops in
 * IEEE double, one candidate per OpenMP iteration, fixed summation orders.
 *
 * Paper: Willemsen, van Nieuwpoort, van Werkhoven, "Bayesian Optimization for
 * auto-tuning GPU kernels" (arXiv 2111.14991).  Readings of points the paper
 * leaves open are noted where they are used.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS 2.220446049250313e-16 /* 2^-52 */

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Section III-D.1: numerical parameters are normalized linearly.  Each
 * parameter's ordered value list is mapped to evenly spaced points of [0, 1]
 * (level i of k -> i / (k - 1)), which removes the distortion of non-linear
 * value lists such as powers of two that the section describes. */
int orc_normalize_grid(int32_t d, const int32_t* levels, int64_t N, const int64_t* cand, double* X) {
  if (d <= 0 || N < 0 || levels == NULL || (N > 0 && X == NULL)) return ORC_E_INVALID_ARG;
  int64_t total = 1;
  for (int32_t j = 0; j < d; ++j) {
    if (levels[j] < 1) return ORC_E_INVALID_ARG;
    if (total > INT64_MAX / levels[j]) return ORC_E_INVALID_ARG;
    total *= levels[j];
  }
  for (int64_t c = 0; c < N; ++c) {
    int64_t g = cand ? cand[c] : c;
    if (g < 0 || g >= total) return ORC_E_INVALID_ARG;
    for (int32_t j = d - 1; j >= 0; --j) {
      int64_t k = levels[j];
      int64_t i = g % k;
      g /= k;
      X[c * d + j] = (k > 1) ? (double)i / (double)(k - 1) : 0.0;
    }
  }
  return ORC_OK;
}

/* Section III-B: Matern covariance at the half-integer orders nu = 3/2 and
 * nu = 5/2, where it reduces to an exponential times a polynomial.  The scaled
 * distance is rho = sqrt(2 nu) r / l (the printed square root over "2 nu r" is
 * read as a typesetting slip: with it the quadratic term of the nu = 5/2 form
 * would not be the square of the linear one). */
double orc_matern(int32_t nu2, double r, double l) {
  if (nu2 == 5) {
    double rho = sqrt(5.0) * r / l;
    return (1.0 + rho + rho * rho / 3.0) * exp(-rho);
  }
  double rho = sqrt(3.0) * r / l;
  return (1.0 + rho) * exp(-rho);
}

/* Euclidean distance in the normalized coordinates (one isotropic lengthscale,
 * Section III-B), by direct differences. */
static double orc_dist(const double* a, const double* b, int32_t d) {
  double s = 0.0;
  for (int32_t t = 0; t < d; ++t) {
    double diff = a[t] - b[t];
    s += diff * diff;
  }
  return sqrt(s);
}

static int orc_gp_ok(const orc_gp* gp) {
  if (gp == NULL) return 0;
  if (gp->nu2 != 3 && gp->nu2 != 5) return 0;
  if (!(gp->lengthscale > 0.0) || !isfinite(gp->lengthscale)) return 0;
  if (!(gp->amp > 0.0) || !isfinite(gp->amp)) return 0;
  if (!(gp->noise >= 0.0) || !isfinite(gp->noise)) return 0;
  if (gp->jitter_tries < 1 || gp->jitter_tries > 20) return 0;
  return 1;
}

/* Diagonal addition for attempt t: the observation noise first, then a
 * tenfold escalation from max(noise, 1e-10 * amp).  The paper fixes no noise
 * or jitter rule; this one keeps a numerically singular K_nn usable. */
static double orc_jitter(const orc_gp* gp, int32_t t) {
  if (t == 0) return gp->noise;
  double base = gp->noise > 1e-10 * gp->amp ? gp->noise : 1e-10 * gp->amp;
  double p = 1.0;
  for (int32_t i = 0; i < t; ++i) p *= 10.0;
  return base * p;
}

/* Cholesky-Banachiewicz factorization of A = K + delta I, row by row, inner
 * sums in increasing k.  A pivot is accepted when it is finite and exceeds
 * n * 2^-52 times the diagonal entry it came from. */
static int orc_cholesky(int32_t n, const double* K, double delta, double* L) {
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j = 0; j <= i; ++j) {
      double a = K[(int64_t)i * n + j] + (i == j ? delta : 0.0);
      double s = a;
      for (int32_t k = 0; k < j; ++k) s -= L[(int64_t)i * n + k] * L[(int64_t)j * n + k];
      if (i == j) {
        if (!isfinite(s) || !(s > (double)n * ORC_EPS * a)) return 0;
        L[(int64_t)i * n + i] = sqrt(s);
      } else {
        L[(int64_t)i * n + j] = s / L[(int64_t)j * n + j];
      }
    }
    for (int32_t j = i + 1; j < n; ++j) L[(int64_t)i * n + j] = 0.0;
  }
  return 1;
}

/* Section III-B with a fixed lengthscale (no hyperparameter search): the fit is
 * the covariance of the observations, its Cholesky factor and
 * alpha = K_nn^-1 (y - m).  The prior mean m is the mean of the observations
 * (Section III-B calls a zero mean usual; positive run times would make every
 * unexplored point look optimal under a zero mean).  f_best = min y is the
 * incumbent f(x+) of Section III-C. */
int orc_fit(int32_t n, int32_t d, const double* Xo, const double* y, const orc_gp* gp,
            double* L, double* alpha, double* mean_y, double* f_best, double* jitter) {
  if (n < 1) return ORC_E_STATE;
  if (d < 1 || Xo == NULL || y == NULL || L == NULL || alpha == NULL) return ORC_E_INVALID_ARG;
  if (!orc_gp_ok(gp)) return ORC_E_INVALID_ARG;
  for (int32_t i = 0; i < n; ++i)
    if (!isfinite(y[i])) return ORC_E_INVALID_ARG;

  double m = 0.0;
  for (int32_t i = 0; i < n; ++i) m += y[i];
  m /= (double)n;
  double fb = y[0];
  for (int32_t i = 1; i < n; ++i)
    if (y[i] < fb) fb = y[i];

  double* K = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  if (K == NULL || z == NULL) {
    free(K);
    free(z);
    return ORC_E_INVALID_ARG;
  }
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = 0; j < n; ++j)
      K[(int64_t)i * n + j] = gp->amp * orc_matern(gp->nu2, orc_dist(Xo + (int64_t)i * d, Xo + (int64_t)j * d, d), gp->lengthscale);

  int ok = 0;
  double delta = 0.0;
  for (int32_t t = 0; t < gp->jitter_tries && !ok; ++t) {
    delta = orc_jitter(gp, t);
    ok = orc_cholesky(n, K, delta, L);
  }
  free(K);
  if (!ok) {
    free(z);
    return ORC_E_NOT_PD;
  }
  /* L z = y - m, then L^T alpha = z. */
  for (int32_t i = 0; i < n; ++i) {
    double s = y[i] - m;
    for (int32_t k = 0; k < i; ++k) s -= L[(int64_t)i * n + k] * z[k];
    z[i] = s / L[(int64_t)i * n + i];
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    double s = z[i];
    for (int32_t k = i + 1; k < n; ++k) s -= L[(int64_t)k * n + i] * alpha[k];
    alpha[i] = s / L[(int64_t)i * n + i];
  }
  free(z);
  if (mean_y) *mean_y = m;
  if (f_best) *f_best = fb;
  if (jitter) *jitter = delta;
  return ORC_OK;
}

/* GP posterior at one point (Section III-B; exhaustive prediction of Section
 * III-G): mu = m + k*^T alpha, var = amp - |v|^2 with L v = k*, clamped at 0.
 * The variance is that of the latent function (no noise term). */
static void orc_predict_one(const double* p, int32_t d, int32_t n, const double* Xo,
                            const double* L, const double* alpha, double mean_y,
                            const orc_gp* gp, double* k, double* v, double* mu, double* var) {
  for (int32_t i = 0; i < n; ++i)
    k[i] = gp->amp * orc_matern(gp->nu2, orc_dist(p, Xo + (int64_t)i * d, d), gp->lengthscale);
  double m = mean_y;
  for (int32_t i = 0; i < n; ++i) m += k[i] * alpha[i];
  double q = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double s = k[i];
    for (int32_t j = 0; j < i; ++j) s -= L[(int64_t)i * n + j] * v[j];
    v[i] = s / L[(int64_t)i * n + i];
    q += v[i] * v[i];
  }
  double s2 = gp->amp - q;
  *mu = m;
  *var = s2 > 0.0 ? s2 : 0.0;
}

void orc_predict(int64_t M, int32_t d, const double* P, int32_t n, const double* Xo,
                 const double* L, const double* alpha, double mean_y, const orc_gp* gp,
                 double* mu, double* var) {
#pragma omp parallel
  {
    double* k = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(static)
    for (int64_t c = 0; c < M; ++c)
      orc_predict_one(P + c * d, d, n, Xo, L, alpha, mean_y, gp, k, v, mu + c, var + c);
    free(k);
    free(v);
  }
}

/* Section III-C, minimization forms, with one exploration offset lambda.
 * tau = f(x+) - lambda; z = (tau - mu) / sigma.
 *   PI  = P(g <= tau) = Phi(z), with Phi(z) = erfc(-z / sqrt 2) / 2;
 *   EI  = E[max(tau - g, 0)] = (tau - mu) Phi(z) + sigma phi(z);
 *   LCB = mu - lambda sigma.
 * The printed PI adds lambda to f(x+); under minimization that would reward
 * exploitation, so the offset is read as subtracted (the usual xi offset).  At
 * sigma = 0 the sigma -> 0 limits are used. */
void orc_acquisitions(double mu, double var, double f_best, double lambda, double* out) {
  double tau = f_best - lambda;
  double sigma = sqrt(var);
  double ei, pi;
  if (sigma > 0.0) {
    double z = (tau - mu) / sigma;
    double Phi = 0.5 * erfc(-z * 0.70710678118654752440);
    double phi = exp(-0.5 * z * z) * 0.39894228040143267794;
    pi = Phi;
    ei = (tau - mu) * Phi + sigma * phi;
  } else {
    ei = tau - mu > 0.0 ? tau - mu : 0.0;
    pi = tau > mu ? 1.0 : (tau == mu ? 0.5 : 0.0);
  }
  out[0] = ei;
  out[1] = pi;
  out[2] = mu - lambda * sigma;
}

/* EI, PI, LCB of every candidate with mask[c] == 0 (rows of out, N x 3);
   NaN rows elsewhere.  The per-point definition is orc_acquisitions. */
void orc_acquisitions_all(int64_t N, const double* mu, const double* var, const uint8_t* mask,
                          double f_best, double lambda, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    if (mask[c]) {
      out[3 * c] = out[3 * c + 1] = out[3 * c + 2] = NAN;
    } else {
      orc_acquisitions(mu[c], var[c], f_best, lambda, out + 3 * c);
    }
  }
}

#define ORC_BLOCK 4096

int orc_step(int64_t N, int32_t d, const double* X, const uint8_t* invalid,
             const uint8_t* visited, int32_t n, const int64_t* obs_idx, const double* y,
             const orc_gp* gp, const orc_acq* acq, double* mu, double* var,
             orc_result* res) {
  if (res == NULL) return ORC_E_INVALID_ARG;
  memset(res, 0, sizeof(*res));
  for (int a = 0; a < 3; ++a) {
    res->idx[a] = -1;
    res->score[a] = NAN;
  }
  res->lambda = NAN;
  res->var_mean = NAN;
  res->jitter = NAN;
#define ORC_FAIL(code) do { res->status = (code); return (code); } while (0)
  if (N < 0 || d < 1 || X == NULL || invalid == NULL || visited == NULL) ORC_FAIL(ORC_E_INVALID_ARG);
  if (n < 1) ORC_FAIL(ORC_E_STATE);
  if (obs_idx == NULL || y == NULL || acq == NULL || !orc_gp_ok(gp)) ORC_FAIL(ORC_E_INVALID_ARG);
  if (acq->mode != 0 && acq->mode != 1) ORC_FAIL(ORC_E_INVALID_ARG);
  for (int32_t i = 0; i < n; ++i)
    if (obs_idx[i] < 0 || obs_idx[i] >= N || invalid[obs_idx[i]]) ORC_FAIL(ORC_E_INVALID_ARG);

  double* Xo = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
  double* L = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* alpha = (double*)malloc(sizeof(double) * (size_t)n);
  double* muw = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* varw = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  int rc = ORC_OK;
  if (!Xo || !L || !alpha || !muw || !varw) {
    rc = ORC_E_INVALID_ARG;
    goto done;
  }
  for (int32_t i = 0; i < n; ++i) memcpy(Xo + (int64_t)i * d, X + obs_idx[i] * d, sizeof(double) * (size_t)d);

  rc = orc_fit(n, d, Xo, y, gp, L, alpha, &res->mean_y, &res->f_best, &res->jitter);
  if (rc != ORC_OK) goto done;
  if (acq->mode == 1 && !(res->f_best > 0.0 && acq->mu_s > 0.0)) {
    rc = ORC_E_INVALID_ARG;
    goto done;
  }

  /* Section III-D.2: predictions only for candidates that are neither
   * restriction-pruned nor already evaluated. */
#pragma omp parallel
  {
    double* k = (double*)malloc(sizeof(double) * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
      if (invalid[c] || visited[c]) {
        muw[c] = NAN;
        varw[c] = NAN;
      } else {
        orc_predict_one(X + c * d, d, n, Xo, L, alpha, res->mean_y, gp, k, v, muw + c, varw + c);
      }
    }
    free(k);
    free(v);
  }

  /* Mean posterior variance over the predicted candidates: per block of 4096
   * candidates in index order, then the block sums in order. */
  {
    int64_t nu = 0;
    double total = 0.0;
    for (int64_t b0 = 0; b0 < N; b0 += ORC_BLOCK) {
      int64_t b1 = b0 + ORC_BLOCK < N ? b0 + ORC_BLOCK : N;
      double part = 0.0;
      for (int64_t c = b0; c < b1; ++c)
        if (!(invalid[c] || visited[c])) {
          part += varw[c];
          ++nu;
        }
      total += part;
    }
    res->n_unmasked = nu;
    if (nu == 0) {
      rc = ORC_E_NO_CANDIDATE;
      goto done;
    }
    res->var_mean = total / (double)nu;
  }

  /* Section III-F: lambda is either the constant or
   * (var_mean / (mu_s / f_best)) / var_s_mean, where var_s_mean is the mean
   * variance after the initial sample (this step's, when none is given). */
  if (acq->mode == 0) {
    res->lambda = acq->lambda_const;
  } else {
    double vs = acq->var_s_mean > 0.0 ? acq->var_s_mean : res->var_mean;
    res->lambda = (res->var_mean / (acq->mu_s / res->f_best)) / vs;
  }

  /* Arg-optimum in increasing original index with strict comparisons: ties
   * keep the lowest index; NaN scores are never chosen. */
  {
    double best[3] = {0.0, 0.0, 0.0};
    for (int64_t c = 0; c < N; ++c) {
      if (invalid[c] || visited[c]) continue;
      double a[3];
      orc_acquisitions(muw[c], varw[c], res->f_best, res->lambda, a);
      for (int q = 0; q < 3; ++q) {
        if (isnan(a[q])) {
          res->nan_seen = 1;
          continue;
        }
        int better;
        if (res->idx[q] < 0) better = 1;
        else if (q < 2) better = a[q] > best[q];
        else better = a[q] < best[q];
        if (better) {
          best[q] = a[q];
          res->idx[q] = c;
        }
      }
    }
    for (int q = 0; q < 3; ++q) res->score[q] = res->idx[q] >= 0 ? best[q] : NAN;
    if (res->nan_seen) rc = ORC_E_NUMERIC;
  }

done:
  if (rc == ORC_OK || rc == ORC_E_NUMERIC) {
    if (mu) memcpy(mu, muw, sizeof(double) * (size_t)N);
    if (var) memcpy(var, varw, sizeof(double) * (size_t)N);
  }
  free(Xo);
  free(L);
  free(alpha);
  free(muw);
  free(varw);
  res->status = rc;
  return rc;
#undef ORC_FAIL
}
