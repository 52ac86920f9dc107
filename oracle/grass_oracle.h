/* GRASS oracle (test infrastructure only): declarations for grass_oracle.c.
 * This header belongs to the oracle alone; the GPU library never includes it. */
#ifndef GRASS_ORACLE_H
#define GRASS_ORACLE_H
#include <stdint.h>

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_ERR_INVALID = -1, ORC_ERR_DISCONNECTED = -2 };

typedef struct {
    double sigma2;      /* target relative condition number (eq. 5: kappa <= sigma^2) */
    int32_t k, t;       /* random vectors, power steps (eqs. 29, 55) */
    uint64_t seed;
    int32_t max_iters;  /* densification passes */
    double budget_frac; /* per-pass budget floor(budget_frac n); 0 = no limit */
    int32_t sim_hops;   /* similarity marks: -1 off, 0 endpoints, 1 endpoints + neighbours */
    int32_t lambda_steps;
    double pcg_rtol;
    int32_t pcg_max_iters;
} orc_opts;

typedef struct {
    int64_t pass;
    double lambda_max, lambda_min, kappa, theta, heat_max;
    int64_t m_off, candidates, accepted, added_total;
    int64_t pcg_iters;
    double pcg_resid;
} orc_pass_stats;

typedef struct {
    double lambda_max, lambda_min, kappa, heat_max, pcg_resid;
    int32_t passes;
    int64_t tree_edges, added_edges, scored_edges;
} orc_summary;

int orc_validate(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w);
int64_t orc_max_spanning_tree(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                              uint8_t *mask);
void orc_laplacian_apply(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                         const uint8_t *use, int k, const double *x, double *y);
void orc_weighted_degree(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                         const uint8_t *use, double *deg);
int orc_root_tree(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                  const uint8_t *tree, int64_t root, int64_t *parent, double *pw, int64_t *order);
void orc_tree_solve(int64_t n, const int64_t *parent, const double *pw, const int64_t *order, int k,
                    const double *b, double *x);
int orc_pcg(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w, const uint8_t *inP,
            const int64_t *parent, const double *pw, const int64_t *order, int k, const double *b, double *x,
            double rtol, int maxit, double *resid);
int orc_sdd_solve(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                  const uint8_t *inP, int p_is_tree, const int64_t *parent, const double *pw,
                  const int64_t *order, int k, const double *b, double *x, double rtol, int maxit,
                  double rtol_inner, double *resid);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void orc_gauss_vectors(int64_t n, int k, uint64_t seed, int64_t pass, double *h0);
int orc_embed(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w, const uint8_t *inP,
              int k, int t, int lambda_steps, uint64_t seed, int64_t pass, double pcg_rtol, int pcg_maxit,
              double *heat, orc_pass_stats *st);
double orc_theta(double sigma2, double lambda_min, double lambda_max, int t);
int64_t orc_filter_select(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *heat,
                          uint8_t *inP, double theta, double heat_max, int sim_hops, int64_t budget,
                          int64_t *ncand);
int orc_sparsify(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                 const orc_opts *o, const uint8_t *init_mask, uint8_t *mask, double *scores, orc_summary *sum,
                 orc_pass_stats *trace, int trace_cap);
int64_t orc_low_stretch_tree(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                             uint64_t seed, int class_bits, int max_rounds, uint8_t *mask, int64_t *cluster);
double orc_tree_stretch(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                        const uint8_t *tree, double *stretch);
#endif
