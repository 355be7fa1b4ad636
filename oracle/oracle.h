/* FP64 CPU oracle for one Bayesian-optimization surrogate step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, constant or helper with the GPU library.
 *
 * What it computes (Willemsen, van Nieuwpoort, van Werkhoven, "Bayesian
 * Optimization for auto-tuning GPU kernels", arXiv 2111.14991):
 *   - the discrete, linearly normalized search space (Section III-D.1) with
 *     restriction-pruned and already-evaluated points excluded (Section III-D.2);
 *   - a Gaussian-process surrogate with a constant mean and a fixed-lengthscale
 *     Matern covariance, nu = 3/2 or 5/2 (Section III-B);
 *   - exhaustive prediction of every remaining point (Section III-G);
 *   - PI, EI and LCB in their minimization form (Section III-C) with either a
 *     constant exploration factor or the contextual-variance factor of
 *     Section III-F;
 *   - the arg-optimum of each acquisition.
 * Every value is computed in IEEE double with a fixed evaluation order, so the
 * results do not depend on the OpenMP thread count.
 */
#ifndef BO_ORACLE_H
#define BO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_INVALID_ARG = 1,
  ORC_E_NOT_PD = 2,
  ORC_E_NO_CANDIDATE = 3,
  ORC_E_STATE = 6,
  ORC_E_NUMERIC = 8
};

typedef struct {
  int32_t nu2;          /* 3 or 5: Matern smoothness nu = nu2 / 2 */
  double lengthscale;   /* l > 0 */
  double amp;           /* prior variance k(0) > 0 */
  double noise;         /* added to the diagonal of K_nn, >= 0 */
  int32_t jitter_tries; /* >= 1 */
} orc_gp;

typedef struct {
  int32_t mode;         /* 0: constant exploration factor, 1: contextual variance */
  double lambda_const;  /* used in mode 0 */
  double mu_s;          /* initial-sample mean (mode 1) */
  double var_s_mean;    /* mean posterior variance after the initial sample (mode 1);
                           <= 0 means "this is that first step" */
} orc_acq;

typedef struct {
  int64_t idx[3];       /* argmax EI, argmax PI, argmin LCB (original indices), -1 if none */
  double score[3];      /* EI, PI, LCB at those indices */
  double lambda;
  double var_mean;
  double jitter;        /* accepted diagonal addition */
  double f_best;
  double mean_y;
  int64_t n_unmasked;
  int32_t status;
  int32_t nan_seen;
} orc_result;

/* Normalized coordinates of candidates given by grid index (row-major, last
 * parameter fastest): x_j = i_j / (k_j - 1), 0 for a one-level parameter.
 * cand == NULL means candidate c is grid point c.  X is N x d row-major. */
int orc_normalize_grid(int32_t d, const int32_t* levels, int64_t N, const int64_t* cand, double* X);

/* Matern correlation at distance r (unit amplitude). */
double orc_matern(int32_t nu2, double r, double l);

/* Fit on n observations.  Xo is n x d, y has n entries.  L (n x n row-major,
 * lower triangle written, upper zeroed) and alpha (n) are outputs. */
int orc_fit(int32_t n, int32_t d, const double* Xo, const double* y, const orc_gp* gp,
            double* L, double* alpha, double* mean_y, double* f_best, double* jitter);

/* Posterior mean and latent variance at M points P (M x d) from a fit. */
void orc_predict(int64_t M, int32_t d, const double* P, int32_t n, const double* Xo,
                 const double* L, const double* alpha, double mean_y, const orc_gp* gp,
                 double* mu, double* var);

/* Acquisition values at one point: out[0] = EI, out[1] = PI, out[2] = LCB. */
void orc_acquisitions(double mu, double var, double f_best, double lambda, double* out);

/* orc_acquisitions at every candidate with mask[c] == 0 (row c of out, N x 3);
 * NaN rows where mask[c] != 0. */
void orc_acquisitions_all(int64_t N, const double* mu, const double* var, const uint8_t* mask,
                          double f_best, double lambda, double* out);

/* One whole step over N candidates X (N x d).  invalid[c] != 0 marks a
 * restriction-pruned candidate, visited[c] != 0 an evaluated one (either way
 * it is excluded from prediction and from the arg-optimum).  obs_idx/y are the
 * n valid observations (indices into the candidate enumeration; an index of an
 * invalid candidate is an error).  mu/var (nullable, N entries) receive the
 * posterior; excluded entries are set to NaN. */
int orc_step(int64_t N, int32_t d, const double* X, const uint8_t* invalid,
             const uint8_t* visited, int32_t n, const int64_t* obs_idx, const double* y,
             const orc_gp* gp, const orc_acq* acq, double* mu, double* var,
             orc_result* res);

/* Number of OpenMP threads the oracle uses. */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
