
/* Declarations shared by the oracle's own C files (test infrastructure only;
 * never included by the GPU library). */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include <stdint.h>

void orc_draw_words(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                    uint32_t p, uint32_t *w);
double orc_u53(uint32_t a, uint32_t b);
void orc_normal2(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                 uint32_t p, double *z);
double orc_gamma(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t jbase,
                 uint32_t p, double shape, int *fail);
double orc_max(const double *x, int64_t n);
void orc_normalise(const double *lw, int64_t n, double *out);
int orc_resample_flag(double ess, int64_t n, double threshold);
int orc_resample(int scheme, uint64_t seed, uint32_t t, uint32_t p, const double *lw,
                 int64_t n, int32_t *anc, double *S_out, double *u_out);

enum {
    ORC_TAG_INIT = 1,
    ORC_TAG_PF_MOVE = 2,
    ORC_TAG_MH_MU = 3,
    ORC_TAG_MH_ETA = 4,
    ORC_TAG_MH_Z = 5,
    ORC_TAG_MH_ACCEPT = 6,
    ORC_TAG_RESAMPLE = 7
};

/* Neumaier compensated sum, added to in index order. */
typedef struct {
    double s, c;
} orc_ksum;

static inline void orc_ks_add(orc_ksum *k, double x)
{
    double t = k->s + x;
    double as = k->s < 0 ? -k->s : k->s, ax = x < 0 ? -x : x;
    if (as >= ax)
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static inline double orc_ks_val(const orc_ksum *k) { return k->s + k->c; }

#endif
