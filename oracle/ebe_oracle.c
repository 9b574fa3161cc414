/*
 * O2: plain FP64 element-by-element Galerkin entries (test infrastructure only).
 *
 * A_ij = -(1/2pi) sum_{a=0..p} sum_{b=0..p} int_{e1} int_{e2} B_i(s) J(s) ln|f(s)-f(t)| B_j(t) J(t) dt ds,
 * with e1 = i+a, e2 = j+b (mod N) the elements of supp B_i, supp B_j: eq. elbyelint,
 * evaluated entry by entry, as the element-by-element cost model of Section 5 counts it.
 *
 *  far pairs  (e2 not in {e1-1, e1, e1+1} mod N): G x G tensor Gauss-Legendre;
 *  near pairs (coincident / adjacent, wrap pair included, t* = t unwrapped next to s):
 *     ln|f(s)-f(t)| = [ln|f(s)-f(t)| - ln|s-t*|] + ln|s-t*|   (kernel split of Section 3.1),
 *     regular bracket: Gn x Gn Gauss (diagonal limit ln J(s), eq. F1_lim),
 *     log part: B J interpolated at Gs Gauss points per element, integrated exactly
 *     with the reference matrices h^2 (ln h w_a w_b + Mhat_ab).
 *
 * B_i(s) on element e1 = i + a is M_p(a + u), u in [0,1) the local coordinate,
 * M_p the cardinal B-spline from the Cox-de Boor recurrence.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double cardinal(int p, double x)
{
    double B[32];
    for (int k = 0; k <= p; ++k) B[k] = (x >= k && x < k + 1) ? 1.0 : 0.0;
    for (int r = 1; r <= p; ++r)
        for (int k = 0; k <= p - r; ++k)
            B[k] = (x - k) / r * B[k] + (k + r + 1 - x) / r * B[k + 1];
    return B[0];
}

typedef struct {
    int p, N;
    int G;  const double *gu, *gw, *gx, *gy, *gJ;   /* far rule; geometry at N*G points  */
    int Gn; const double *nu, *nw, *nx, *ny, *nJ;   /* near regular part; N*Gn points    */
    int Gs; const double *su, *sw, *sJ;             /* near log part; J at N*Gs points   */
    const double *Mco, *Madj;                       /* Gs x Gs reference matrices        */
} problem;

static double pair_far(const problem *P, int e1, int a, int e2, int b)
{
    const int G = P->G;
    const double h = 1.0 / P->N;
    double acc = 0.0;
    for (int g1 = 0; g1 < G; ++g1) {
        const int k1 = e1 * G + g1;
        const double phi1 = P->gw[g1] * cardinal(P->p, a + P->gu[g1]) * P->gJ[k1];
        for (int g2 = 0; g2 < G; ++g2) {
            const int k2 = e2 * G + g2;
            const double phi2 = P->gw[g2] * cardinal(P->p, b + P->gu[g2]) * P->gJ[k2];
            const double dx = P->gx[k1] - P->gx[k2], dy = P->gy[k1] - P->gy[k2];
            acc += phi1 * log(sqrt(dx * dx + dy * dy)) * phi2;
        }
    }
    return h * h * acc;
}

/* dd = unwrapped offset of e2 relative to e1: -1, 0 or +1 */
static double pair_near(const problem *P, int e1, int a, int e2, int b, int dd)
{
    const double h = 1.0 / P->N;
    double reg = 0.0;
    for (int g1 = 0; g1 < P->Gn; ++g1) {
        const int k1 = e1 * P->Gn + g1;
        const double phi1 = P->nw[g1] * cardinal(P->p, a + P->nu[g1]) * P->nJ[k1];
        for (int g2 = 0; g2 < P->Gn; ++g2) {
            const int k2 = e2 * P->Gn + g2;
            const double phi2 = P->nw[g2] * cardinal(P->p, b + P->nu[g2]) * P->nJ[k2];
            double bracket;
            if (dd == 0 && g1 == g2) {
                bracket = log(P->nJ[k1]);
            } else {
                const double dx = P->nx[k1] - P->nx[k2], dy = P->ny[k1] - P->ny[k2];
                const double st = h * fabs(P->nu[g1] - P->nu[g2] - dd);
                bracket = log(sqrt(dx * dx + dy * dy)) - log(st);
            }
            reg += phi1 * bracket * phi2;
        }
    }
    const int Gs = P->Gs;
    double sing = 0.0;
    const double lnh = log(h);
    for (int al = 0; al < Gs; ++al) {
        const double phi1 = cardinal(P->p, a + P->su[al]) * P->sJ[e1 * Gs + al];
        for (int be = 0; be < Gs; ++be) {
            const double phi2 = cardinal(P->p, b + P->su[be]) * P->sJ[e2 * Gs + be];
            double m;
            if (dd == 0)      m = P->Mco[al * Gs + be];
            else if (dd == 1) m = P->Madj[al * Gs + be];
            else              m = P->Madj[be * Gs + al];
            sing += phi1 * phi2 * (lnh * P->sw[al] * P->sw[be] + m);
        }
    }
    return h * h * (reg + sing);
}

static double entry(const problem *P, int i, int j)
{
    const int N = P->N, p = P->p;
    double acc = 0.0;
    for (int a = 0; a <= p; ++a) {
        const int e1 = (i + a) % N;
        for (int b = 0; b <= p; ++b) {
            const int e2 = (j + b) % N;
            const int d = ((e2 - e1) % N + N) % N;
            if (d == 0)          acc += pair_near(P, e1, a, e2, b, 0);
            else if (d == 1)     acc += pair_near(P, e1, a, e2, b, 1);
            else if (d == N - 1) acc += pair_near(P, e1, a, e2, b, -1);
            else                 acc += pair_far(P, e1, a, e2, b);
        }
    }
    return -acc / (2.0 * M_PI);
}

/* out[k] = A_{ii[k], jj[k]} for k < n; returns the number of threads used. */
int oracle_ebe_entries(int p, int N,
                       int G, const double *gu, const double *gw,
                       const double *gx, const double *gy, const double *gJ,
                       int Gn, const double *nu, const double *nw,
                       const double *nx, const double *ny, const double *nJ,
                       int Gs, const double *su, const double *sw, const double *sJ,
                       const double *Mco, const double *Madj,
                       int64_t n, const int32_t *ii, const int32_t *jj, double *out, int nthreads)
{
    problem P = {p, N, G, gu, gw, gx, gy, gJ, Gn, nu, nw, nx, ny, nJ, Gs, su, sw, sJ, Mco, Madj};
    int used = 1;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n; ++k) out[k] = entry(&P, ii[k], jj[k]);
    }
#else
    (void)nthreads;
    for (int64_t k = 0; k < n; ++k) out[k] = entry(&P, ii[k], jj[k]);
#endif
    return used;
}
