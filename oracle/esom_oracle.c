/*
 * Plain FP64 CPU EmbedSOM oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the reference that the GPU library is checked against.  It is
 * deliberately slow and literal: every distance is a direct difference in
 * double precision, neighbours come from a plain sorted insertion, and the
 * 2x2 system is accumulated pair by pair in the order the method states.
 * It shares no code, header, table or constant with the GPU library and
 * must only be called from tests/, the smoke check and the CPU-baseline leg
 * of the benchmark.
 *
 * Method (Section "Landmark-directed dimensionality reduction" of the paper,
 * the four numbered steps of its EmbedSOM description):
 *   1. the k nearest landmarks of X_i in L (3 <= k <= g), Euclidean distance;
 *   2. a smooth rank-ordered score: highest for the closest landmark and zero
 *      for the k-th one when k < g;
 *   3. for every pair (u,v) of neighbours, D_uv(X_i) = affine coordinate of
 *      X_i projected on the line with 0 at L_u and 1 at L_v, and the matching
 *      2-D affine coordinate d_uv(p) on the line l_u -> l_v;
 *   4. x_i = argmin_p sum_{u<v} s_u s_v (D_uv - d_uv(p))^2, which is a 2x2
 *      linear system solved by Cramer's rule (Section "Projection step").
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - score formula (step 2): the paper defers it to the original EmbedSOM
 *     publication.  With rank weights w_i = 1/i, W = sum w_i, the weighted
 *     mean mu and variance sigma^2 of the neighbour distances delta_i,
 *       e_i = exp(boost * (mu - delta_i) / sigma)       (e_i = 1 if the
 *             variance is <= 1e-30 mu^2),
 *       c_i = 1 - exp(cutoff * (delta_i / delta_k - 1)) when k < g, else 1,
 *       s_i = e_i * c_i.
 *   - pair weight exponent `adjust` (a): the pair (u,v) enters the objective
 *     with weight s_u s_v |h|^(2-2a), h = l_v - l_u.  a = 1 is the paper's
 *     objective exactly.
 *   - a tiny "gravity" term eps * sum_i s_i |p - l_{n_i}|^2 keeps the system
 *     non-singular (k = 3 leaves a rank-one system otherwise).
 *   - pairs whose HD or 2-D landmarks coincide exactly are skipped.
 *   - degenerate neighbourhoods (all delta equal, sum of scores zero, or a
 *     numerically singular system, det <= 1e-9 (tr/2)^2) map to the centroid
 *     of the neighbours' 2-D positions.  A rank-deficient system (k = 3
 *     without gravity, or collinear 2-D neighbours) has det = 0 exactly, but
 *     its computed det is rounding noise of either sign; the relative bound
 *     makes the decision independent of the summation order.
 *   - ties between equal distances break by landmark index.
 *
 * Landmark update (Section "User supervision and model interaction"): one
 * batch step of k-means (graph mode) or of a batch SOM over the 2-D landmark
 * topology (SOM mode), blended into L with learning rate alpha.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* ---- step 1: k nearest landmarks by (squared distance, index) ---------- */

/* Squared Euclidean distance between a point and a landmark, as a plain sum
 * of squared coordinate differences in double. */
static double sqdist(const float *x, const float *y, int d)
{
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = (double)x[t] - (double)y[t];
        s += diff * diff;
    }
    return s;
}

/* Lexicographic order on (distance, index). */
static int before(double da, int ia, double db, int ib)
{
    return da < db || (da == db && ia < ib);
}

/* Keeps the m smallest (distance, index) pairs of one point, sorted
 * ascending, by plain insertion over all g landmarks.  Slots that stay empty
 * (m > g) hold index -1 and distance +inf. */
static void nearest_m(const float *x, const float *L, int g, int d, int m,
                      int *idx, double *d2)
{
    for (int i = 0; i < m; ++i) {
        idx[i] = -1;
        d2[i] = INFINITY;
    }
    for (int j = 0; j < g; ++j) {
        double dj = sqdist(x, L + (size_t)j * d, d);
        if (idx[m - 1] >= 0 && !before(dj, j, d2[m - 1], idx[m - 1]))
            continue;
        int pos = m - 1;
        while (pos > 0 && (idx[pos - 1] < 0 || before(dj, j, d2[pos - 1], idx[pos - 1]))) {
            idx[pos] = idx[pos - 1];
            d2[pos] = d2[pos - 1];
            --pos;
        }
        idx[pos] = j;
        d2[pos] = dj;
    }
}

/* ---- step 2: scores ------------------------------------------------------ */

/* Scores of k sorted neighbour distances delta[0..k-1] (Euclidean, not
 * squared).  Returns 1 if the neighbourhood is degenerate (all distances
 * equal), 0 otherwise. */
int oracle_scores(const double *delta, int k, int g, double boost, double cutoff,
                  double *s)
{
    if (k < 1)
        return ORACLE_EINVAL;
    if (delta[0] == delta[k - 1]) {
        for (int i = 0; i < k; ++i)
            s[i] = 0.0;
        return 1;
    }
    /* rank weights 1/i; the weighted mean, then the weighted mean of the
     * squared deviations from it (the variance as defined, which keeps its
     * relative accuracy however small the spread of the distances) */
    double W = 0.0, mu = 0.0;
    for (int i = 0; i < k; ++i) {
        double w = 1.0 / (double)(i + 1);
        W += w;
        mu += w * delta[i];
    }
    mu /= W;
    double var = 0.0;
    for (int i = 0; i < k; ++i) {
        double dev = delta[i] - mu;
        var += dev * dev / (double)(i + 1);
    }
    var /= W;
    for (int i = 0; i < k; ++i) {
        double e;
        if (var <= 1e-30 * mu * mu)
            e = 1.0;
        else
            e = exp(boost * (mu - delta[i]) / sqrt(var));
        double c = 1.0;
        if (k < g)
            c = 1.0 - exp(cutoff * (delta[i] / delta[k - 1] - 1.0));
        s[i] = e * c;
    }
    return 0;
}

/* ---- steps 3 and 4 for one point ---------------------------------------- */

typedef struct {
    double boost, adjust, cutoff, gravity;
} oracle_params;

/* Projects one point.  nb[0..k-1] are its neighbours sorted by distance,
 * d2[0..k-1] their squared distances.  Writes p[0..1]; returns 1 if the
 * centroid fallback was taken. */
static int project_point(const float *x, const float *L, const float *l, int g,
                         int d, int k, const int *nb, const double *d2,
                         const oracle_params *P, double *s_scratch,
                         double *delta_scratch, double *p)
{
    for (int i = 0; i < k; ++i)
        delta_scratch[i] = sqrt(d2[i]);
    int degenerate = oracle_scores(delta_scratch, k, g, P->boost, P->cutoff, s_scratch);
    const double *s = s_scratch;

    double ssum = 0.0;
    for (int i = 0; i < k; ++i)
        ssum += s[i];

    /* Normal equations of sum_{u<v} w_uv (D_uv - d_uv(p))^2 with
     * d_uv(p) = <h, p - l_u> / |h|^2: M p = r. */
    double M00 = 0.0, M01 = 0.0, M11 = 0.0, r0 = 0.0, r1 = 0.0;
    if (!degenerate) {
        for (int i = 0; i < k; ++i) {
            int u = nb[i];
            const float *Lu = L + (size_t)u * d;
            double lux = l[2 * u], luy = l[2 * u + 1];
            for (int j = i + 1; j < k; ++j) {
                int v = nb[j];
                const float *Lv = L + (size_t)v * d;
                /* D_uv: coordinate of x on the HD line L_u -> L_v. */
                double HH = 0.0, xH = 0.0;
                for (int t = 0; t < d; ++t) {
                    double H = (double)Lv[t] - (double)Lu[t];
                    HH += H * H;
                    xH += ((double)x[t] - (double)Lu[t]) * H;
                }
                if (HH == 0.0)
                    continue;
                double D = xH / HH;
                double hx = (double)l[2 * v] - lux, hy = (double)l[2 * v + 1] - luy;
                double hh = hx * hx + hy * hy;
                if (hh == 0.0)
                    continue;
                double q = s[i] * s[j] * pow(hh, -P->adjust);
                double rhs = D + (hx * lux + hy * luy) / hh;
                M00 += q * hx * hx / hh;
                M01 += q * hx * hy / hh;
                M11 += q * hy * hy / hh;
                r0 += q * hx * rhs;
                r1 += q * hy * rhs;
            }
        }
        for (int i = 0; i < k; ++i) {
            double gs = P->gravity * s[i];
            M00 += gs;
            M11 += gs;
            r0 += gs * l[2 * nb[i]];
            r1 += gs * l[2 * nb[i] + 1];
        }
    }
    double det = M00 * M11 - M01 * M01;
    double htr = 0.5 * (M00 + M11);
    if (degenerate || ssum == 0.0 || !(det > 1e-9 * htr * htr)) {
        double cx = 0.0, cy = 0.0;
        for (int i = 0; i < k; ++i) {
            cx += l[2 * nb[i]];
            cy += l[2 * nb[i] + 1];
        }
        p[0] = cx / k;
        p[1] = cy / k;
        return 1;
    }
    /* Cramer's rule. */
    p[0] = (r0 * M11 - M01 * r1) / det;
    p[1] = (M00 * r1 - M01 * r0) / det;
    return 0;
}

/* ---- the same four steps with a 3-D output ----------------------------------- */

/* Determinant of a 3 x 3 matrix by cofactor expansion along the first row. */
static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Projects one point into 3-D: the paper states the method in 2-D for
 * brevity (Section "Landmark-directed dimensionality reduction"); with 3-D
 * landmark positions l (g x 3) the same objective sum_{u<v} w_uv (D_uv -
 * d_uv(p))^2 plus gravity has 3 x 3 normal equations M p = r, solved by
 * Cramer's rule.  The singular-system rule scales with the dimension: det <=
 * 1e-9 (tr/3)^3 maps to the centroid of the neighbours' 3-D positions. */
static int project_point3(const float *x, const float *L, const float *l, int g,
                          int d, int k, const int *nb, const double *d2,
                          const oracle_params *P, double *s_scratch,
                          double *delta_scratch, double *p)
{
    for (int i = 0; i < k; ++i)
        delta_scratch[i] = sqrt(d2[i]);
    int degenerate = oracle_scores(delta_scratch, k, g, P->boost, P->cutoff, s_scratch);
    const double *s = s_scratch;
    double ssum = 0.0;
    for (int i = 0; i < k; ++i)
        ssum += s[i];
    double M[3][3] = {{0}}, r[3] = {0};
    if (!degenerate) {
        for (int i = 0; i < k; ++i) {
            int u = nb[i];
            const float *Lu = L + (size_t)u * d;
            const float *lu = l + (size_t)3 * u;
            for (int j = i + 1; j < k; ++j) {
                int v = nb[j];
                const float *Lv = L + (size_t)v * d;
                const float *lv = l + (size_t)3 * v;
                double HH = 0.0, xH = 0.0;
                for (int t = 0; t < d; ++t) {
                    double H = (double)Lv[t] - (double)Lu[t];
                    HH += H * H;
                    xH += ((double)x[t] - (double)Lu[t]) * H;
                }
                if (HH == 0.0)
                    continue;
                double D = xH / HH;
                double h[3], hh = 0.0, hl = 0.0;
                for (int a = 0; a < 3; ++a) {
                    h[a] = (double)lv[a] - (double)lu[a];
                    hh += h[a] * h[a];
                    hl += h[a] * (double)lu[a];
                }
                if (hh == 0.0)
                    continue;
                double q = s[i] * s[j] * pow(hh, -P->adjust);
                double rhs = D + hl / hh;
                for (int a = 0; a < 3; ++a) {
                    for (int b = 0; b < 3; ++b)
                        M[a][b] += q * h[a] * h[b] / hh;
                    r[a] += q * h[a] * rhs;
                }
            }
        }
        for (int i = 0; i < k; ++i) {
            double gs = P->gravity * s[i];
            for (int a = 0; a < 3; ++a) {
                M[a][a] += gs;
                r[a] += gs * l[(size_t)3 * nb[i] + a];
            }
        }
    }
    double det = det3(M);
    double tr3 = (M[0][0] + M[1][1] + M[2][2]) / 3.0;
    if (degenerate || ssum == 0.0 || !(det > 1e-9 * tr3 * tr3 * tr3)) {
        for (int a = 0; a < 3; ++a) {
            double c = 0.0;
            for (int i = 0; i < k; ++i)
                c += l[(size_t)3 * nb[i] + a];
            p[a] = c / k;
        }
        return 1;
    }
    for (int c = 0; c < 3; ++c) {
        double A[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                A[a][b] = (b == c) ? r[a] : M[a][b];
        p[c] = det3(A) / det;
    }
    return 0;
}

/* ---- threaded drivers ------------------------------------------------------ */

typedef struct {
    const float *X, *L, *l;
    int64_t n, ldx;
    int d, g, k, m;
    oracle_params P;
    double *out;   /* n x dim or NULL */
    int dim;       /* output dimension: 2, or 3 (then l is g x 3) */
    int32_t *idx;  /* n x m or NULL */
    double *d2out; /* n x m or NULL */
    int64_t begin, end;
    int64_t n_degenerate;
    int status;
} embed_job;

static void *embed_worker(void *arg)
{
    embed_job *J = (embed_job *)arg;
    int m = J->m;
    int *nb = (int *)malloc(sizeof(int) * (size_t)m);
    double *d2 = (double *)malloc(sizeof(double) * (size_t)m);
    double *s = (double *)malloc(sizeof(double) * (size_t)J->k);
    double *dl = (double *)malloc(sizeof(double) * (size_t)J->k);
    if (!nb || !d2 || !s || !dl) {
        J->status = ORACLE_ENOMEM;
        free(nb); free(d2); free(s); free(dl);
        return NULL;
    }
    for (int64_t i = J->begin; i < J->end; ++i) {
        const float *x = J->X + i * J->ldx;
        nearest_m(x, J->L, J->g, J->d, m, nb, d2);
        if (J->idx)
            for (int t = 0; t < m; ++t)
                J->idx[i * m + t] = nb[t];
        if (J->d2out)
            for (int t = 0; t < m; ++t)
                J->d2out[i * m + t] = d2[t];
        if (J->out && J->dim == 3) {
            double p[3];
            J->n_degenerate += project_point3(x, J->L, J->l, J->g, J->d, J->k, nb, d2,
                                              &J->P, s, dl, p);
            J->out[3 * i] = p[0];
            J->out[3 * i + 1] = p[1];
            J->out[3 * i + 2] = p[2];
        } else if (J->out) {
            double p[2];
            J->n_degenerate += project_point(x, J->L, J->l, J->g, J->d, J->k, nb, d2,
                                             &J->P, s, dl, p);
            J->out[2 * i] = p[0];
            J->out[2 * i + 1] = p[1];
        }
    }
    free(nb); free(d2); free(s); free(dl);
    return NULL;
}

static int run_jobs(embed_job *proto, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (proto->n < nthreads)
        nthreads = proto->n > 0 ? (int)proto->n : 1;
    embed_job *jobs = (embed_job *)calloc((size_t)nthreads, sizeof(embed_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs); free(th);
        return ORACLE_ENOMEM;
    }
    int64_t chunk = (proto->n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].begin = t * chunk < proto->n ? t * chunk : proto->n;
        jobs[t].end = (t + 1) * chunk < proto->n ? (t + 1) * chunk : proto->n;
        jobs[t].n_degenerate = 0;
        jobs[t].status = ORACLE_OK;
    }
    if (nthreads == 1) {
        embed_worker(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; ++t)
            pthread_create(&th[t], NULL, embed_worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t)
            pthread_join(th[t], NULL);
    }
    int status = ORACLE_OK;
    proto->n_degenerate = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status != ORACLE_OK)
            status = jobs[t].status;
        proto->n_degenerate += jobs[t].n_degenerate;
    }
    free(jobs); free(th);
    return status;
}

/* The m nearest landmarks of every point (m may exceed k so that callers can
 * see the (k+1)-th distance), sorted by (squared distance, index). */
int oracle_knn(const float *X, int64_t n, int d, int64_t ldx, const float *L, int g,
               int m, int32_t *idx, double *d2, int nthreads)
{
    if (n < 0 || d < 1 || g < 1 || m < 1 || ldx < d || !X || !L || !idx || !d2)
        return ORACLE_EINVAL;
    embed_job J;
    memset(&J, 0, sizeof J);
    J.X = X; J.L = L; J.n = n; J.ldx = ldx; J.d = d; J.g = g; J.k = m; J.m = m;
    J.idx = idx; J.d2out = d2;
    return run_jobs(&J, nthreads);
}

/* EmbedSOM projection of n points.  out is n x 2 doubles.  idx and d2 (each
 * n x (k+1), may be NULL) receive the k+1 nearest landmarks; the last slot
 * is index -1 / +inf when k == g.  *n_degenerate counts centroid fallbacks. */
int oracle_embed(const float *X, int64_t n, int d, int64_t ldx, const float *L,
                 const float *l, int g, int k, double boost, double adjust,
                 double cutoff, double gravity, double *out, int32_t *idx, double *d2,
                 int64_t *n_degenerate, int nthreads)
{
    if (n < 0 || d < 1 || g < 3 || k < 3 || k > g || ldx < d || !X || !L || !l || !out)
        return ORACLE_EINVAL;
    embed_job J;
    memset(&J, 0, sizeof J);
    J.X = X; J.L = L; J.l = l; J.n = n; J.ldx = ldx; J.d = d; J.g = g; J.k = k;
    J.m = k + 1;
    J.P.boost = boost; J.P.adjust = adjust; J.P.cutoff = cutoff; J.P.gravity = gravity;
    J.out = out; J.dim = 2; J.idx = idx; J.d2out = d2;
    int st = run_jobs(&J, nthreads);
    if (n_degenerate)
        *n_degenerate = J.n_degenerate;
    return st;
}

/* The projection with a 3-D output: l is g x 3, out is n x 3 doubles; other
 * arguments as for oracle_embed. */
int oracle_embed3(const float *X, int64_t n, int d, int64_t ldx, const float *L,
                  const float *l, int g, int k, double boost, double adjust,
                  double cutoff, double gravity, double *out, int32_t *idx, double *d2,
                  int64_t *n_degenerate, int nthreads)
{
    if (n < 0 || d < 1 || g < 3 || k < 3 || k > g || ldx < d || !X || !L || !l || !out)
        return ORACLE_EINVAL;
    embed_job J;
    memset(&J, 0, sizeof J);
    J.X = X; J.L = L; J.l = l; J.n = n; J.ldx = ldx; J.d = d; J.g = g; J.k = k;
    J.m = k + 1;
    J.P.boost = boost; J.P.adjust = adjust; J.P.cutoff = cutoff; J.P.gravity = gravity;
    J.out = out; J.dim = 3; J.idx = idx; J.d2out = d2;
    int st = run_jobs(&J, nthreads);
    if (n_degenerate)
        *n_degenerate = J.n_degenerate;
    return st;
}

/* ---- landmark update --------------------------------------------------------- */

/* One batch landmark-update step.  kind 0: k-means, L_j += alpha (mean_j - L_j)
 * for every landmark that owns at least one point.  kind 1: batch SOM over
 * the 2-D topology, with neighbourhood h_jb = exp(-|l_j - l_b|^2 / (2 sigma^2))
 * (h_jb = [j == b] when sigma == 0):
 *   L_j += alpha (sum_b h_jb S_b / sum_b h_jb c_b - L_j)  when the denominator
 * is positive.  S_b and c_b are the coordinate sums and counts of the points
 * whose nearest landmark is b.  Lout is g x d doubles, counts is g. */
int oracle_landmark_update(const float *X, int64_t n, int d, int64_t ldx,
                           const float *L, const float *l, int g, int kind,
                           double alpha, double sigma, double *Lout, int64_t *counts,
                           int nthreads)
{
    if (n < 0 || d < 1 || g < 1 || ldx < d || !X || !L || !Lout || (kind != 0 && kind != 1))
        return ORACLE_EINVAL;
    if (kind == 1 && (!l || sigma < 0.0))
        return ORACLE_EINVAL;
    int32_t *nearest = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *nd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *S = (double *)calloc((size_t)g * d, sizeof(double));
    double *c = (double *)calloc((size_t)g, sizeof(double));
    if (!nearest || !nd || !S || !c) {
        free(nearest); free(nd); free(S); free(c);
        return ORACLE_ENOMEM;
    }
    int st = ORACLE_OK;
    if (n > 0)
        st = oracle_knn(X, n, d, ldx, L, g, 1, nearest, nd, nthreads);
    if (st == ORACLE_OK) {
        for (int64_t i = 0; i < n; ++i) {
            int b = nearest[i];
            c[b] += 1.0;
            for (int t = 0; t < d; ++t)
                S[(size_t)b * d + t] += (double)X[i * ldx + t];
        }
        for (int j = 0; j < g; ++j) {
            if (counts)
                counts[j] = (int64_t)c[j];
            double den = 0.0;
            double *num = Lout + (size_t)j * d; /* used as accumulator */
            for (int t = 0; t < d; ++t)
                num[t] = 0.0;
            if (kind == 0) {
                den = c[j];
                for (int t = 0; t < d; ++t)
                    num[t] = S[(size_t)j * d + t];
            } else {
                for (int b = 0; b < g; ++b) {
                    double h;
                    if (sigma == 0.0) {
                        h = (b == j) ? 1.0 : 0.0;
                    } else {
                        double dx = (double)l[2 * j] - (double)l[2 * b];
                        double dy = (double)l[2 * j + 1] - (double)l[2 * b + 1];
                        h = exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
                    }
                    den += h * c[b];
                    for (int t = 0; t < d; ++t)
                        num[t] += h * S[(size_t)b * d + t];
                }
            }
            for (int t = 0; t < d; ++t) {
                double Lj = (double)L[(size_t)j * d + t];
                num[t] = den > 0.0 ? Lj + alpha * (num[t] / den - Lj) : Lj;
            }
        }
    }
    free(nearest); free(nd); free(S); free(c);
    return st;
}

/* ---- online SOM training and new-landmark fitting -------------------------- */

/* Supervised SOM training (Section "Supervised training of self-organizing
 * maps"): the 2-D landmarks l are the map topology and the high-dimensional
 * landmarks L are the neuron weights, trained with the user's neighbourhood
 * size sigma and learning rate alpha, which may change from step to step.
 * Kohonen's online rule moves every landmark towards a presented point x by
 * alpha h(j, b) (x - L_j), b the point's best-matching (nearest) landmark and
 * h(j, b) = exp(-|l_j - l_b|^2 / (2 sigma^2)) (h = [j == b] for sigma = 0).
 * One step here presents a batch of B points (rows batch_idx[t*B .. t*B+B-1]
 * of X), finds every point's best-matching landmark against the step's
 * landmarks, and applies the average of the B single-point updates:
 *   L_j <- L_j + (alpha_t / B) sum_i h(j, b_i) (x_i - L_j).
 * With B = 1 this is the serial online rule.  Landmarks with frozen[j] != 0
 * keep their position (they still match points).  The landmarks are stored
 * as float32 between steps, as the caller's array is.  Batch entries outside
 * [0, n) present no point (they still count in B). */
int oracle_som_train(const float *X, int64_t n, int d, int64_t ldx, float *L, const float *l,
                     int g, const int32_t *batch_idx, int B, int T, const double *sigma,
                     const double *alpha, const uint8_t *frozen)
{
    if (n < 0 || d < 1 || g < 1 || B < 1 || T < 0 || ldx < d || !X || !L || !l || !batch_idx ||
        !sigma || !alpha)
        return ORACLE_EINVAL;
    int *bmu = (int *)malloc(sizeof(int) * (size_t)B);
    double *delta = (double *)malloc(sizeof(double) * (size_t)g * d);
    if (!bmu || !delta) {
        free(bmu); free(delta);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < T; ++t) {
        const int32_t *rows = batch_idx + (size_t)t * B;
        /* best-matching landmarks against this step's landmarks */
        for (int i = 0; i < B; ++i) {
            bmu[i] = -1;
            if (rows[i] < 0 || rows[i] >= n)
                continue;
            double d2;
            nearest_m(X + (int64_t)rows[i] * ldx, L, g, d, 1, &bmu[i], &d2);
        }
        /* the average of the single-point updates */
        for (int j = 0; j < g; ++j) {
            double *dj = delta + (size_t)j * d;
            for (int c = 0; c < d; ++c)
                dj[c] = 0.0;
            for (int i = 0; i < B; ++i) {
                int b = bmu[i];
                if (b < 0)
                    continue;
                double h;
                if (sigma[t] == 0.0) {
                    h = (b == j) ? 1.0 : 0.0;
                } else {
                    double dx = (double)l[2 * j] - (double)l[2 * b];
                    double dy = (double)l[2 * j + 1] - (double)l[2 * b + 1];
                    h = exp(-(dx * dx + dy * dy) / (2.0 * sigma[t] * sigma[t]));
                }
                const float *x = X + (int64_t)rows[i] * ldx;
                for (int c = 0; c < d; ++c)
                    dj[c] += h * ((double)x[c] - (double)L[(size_t)j * d + c]);
            }
        }
        for (int j = 0; j < g; ++j) {
            if (frozen && frozen[j])
                continue;
            for (int c = 0; c < d; ++c) {
                double v = (double)L[(size_t)j * d + c] + alpha[t] / (double)B * delta[(size_t)j * d + c];
                L[(size_t)j * d + c] = (float)v;
            }
        }
    }
    free(bmu); free(delta);
    return ORACLE_OK;
}

/* High-dimensional position of a landmark added at 2-D position p (Section
 * "Supervised training of self-organizing maps": fitted from the landmarks
 * that are close in 2-D).  The kfit landmarks nearest to p in 2-D (by
 * (squared distance, index)) get weights w_j = exp(-|l_j - p|^2 / (2 sigma^2)),
 * here scaled by a common factor so that the nearest one weighs 1 (neither the
 * fit nor the mean depends on a common factor, and no weight underflows);
 * an affine map z -> A z + c from 2-D to the high-dimensional space is fitted
 * to them by weighted least squares, min sum_j w_j |L_j - A l_j - c|^2, and
 * evaluated at p.  When the neighbours do not determine an affine map (fewer
 * than three, or collinear: det of the 3 x 3 normal matrix <= 1e-12 times the
 * cube of its mean diagonal), the weighted mean of their L_j is used. */
int oracle_fit_landmarks(const float *L, const float *l, int g, int d, const float *p, int m,
                         int kfit, double sigma, double *out)
{
    if (g < 1 || d < 1 || m < 0 || kfit < 1 || !(sigma > 0.0) || !L || !l || !p || !out)
        return ORACLE_EINVAL;
    if (kfit > g)
        kfit = g;
    int *nb = (int *)malloc(sizeof(int) * (size_t)kfit);
    double *nd = (double *)malloc(sizeof(double) * (size_t)kfit);
    if (!nb || !nd) {
        free(nb); free(nd);
        return ORACLE_ENOMEM;
    }
    for (int q = 0; q < m; ++q) {
        double px = p[2 * q], py = p[2 * q + 1];
        /* the kfit nearest in 2-D, by plain insertion */
        for (int i = 0; i < kfit; ++i) {
            nb[i] = -1;
            nd[i] = INFINITY;
        }
        for (int j = 0; j < g; ++j) {
            double dx = (double)l[2 * j] - px, dy = (double)l[2 * j + 1] - py;
            double dj = dx * dx + dy * dy;
            if (nb[kfit - 1] >= 0 && !before(dj, j, nd[kfit - 1], nb[kfit - 1]))
                continue;
            int pos = kfit - 1;
            while (pos > 0 && (nb[pos - 1] < 0 || before(dj, j, nd[pos - 1], nb[pos - 1]))) {
                nb[pos] = nb[pos - 1];
                nd[pos] = nd[pos - 1];
                --pos;
            }
            nb[pos] = j;
            nd[pos] = dj;
        }
        /* weighted normal equations G a = r of the affine fit, z = (lx, ly, 1) */
        double G[3][3] = {{0}}, W = 0.0;
        for (int i = 0; i < kfit; ++i) {
            double w = exp(-(nd[i] - nd[0]) / (2.0 * sigma * sigma));
            double z[3] = {l[2 * nb[i]], l[2 * nb[i] + 1], 1.0};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    G[a][b] += w * z[a] * z[b];
            W += w;
        }
        double det = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                     G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                     G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
        double md = (G[0][0] + G[1][1] + G[2][2]) / 3.0;
        double *o = out + (size_t)q * d;
        if (kfit >= 3 && det > 1e-12 * md * md * md) {
            /* v = G^{-1} (px, py, 1) by Cramer's rule; the fitted map at p is
             * sum_j w_j (v . z_j) L_j */
            double e[3] = {px, py, 1.0}, v[3];
            for (int c = 0; c < 3; ++c) {
                double M[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        M[a][b] = (b == c) ? e[a] : G[a][b];
                v[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                        M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                        M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
            }
            for (int c = 0; c < d; ++c)
                o[c] = 0.0;
            for (int i = 0; i < kfit; ++i) {
                double w = exp(-(nd[i] - nd[0]) / (2.0 * sigma * sigma));
                double beta = w * (v[0] * l[2 * nb[i]] + v[1] * l[2 * nb[i] + 1] + v[2]);
                for (int c = 0; c < d; ++c)
                    o[c] += beta * (double)L[(size_t)nb[i] * d + c];
            }
        } else {
            for (int c = 0; c < d; ++c)
                o[c] = 0.0;
            for (int i = 0; i < kfit; ++i) {
                double w = exp(-(nd[i] - nd[0]) / (2.0 * sigma * sigma));
                for (int c = 0; c < d; ++c)
                    o[c] += w * (double)L[(size_t)nb[i] * d + c];
            }
            for (int c = 0; c < d; ++c)
                o[c] /= W;
        }
    }
    free(nb); free(nd);
    return ORACLE_OK;
}

/* ---- graph-mode supervision ------------------------------------------------------
 * Section "Semi-supervised structure reconstruction": the high-dimensional
 * landmarks come from an interactive k-means (oracle_landmark_update, kind 0)
 * and their 2-D positions from a simple force-based layout of a neighbourhood
 * graph of L, which the user steers by dragging nodes; landmarks are added by
 * duplicating one in both spaces and removed likewise.  The paper names no
 * graph or force law; the readings below are this build's. */

/* Neighbourhood graph of the landmarks: for every landmark u its kg nearest
 * other landmarks by (squared distance, index), u itself excluded.  nbr and d2
 * are g x kg; slots beyond g - 1 neighbours hold -1 / +inf. */
int oracle_landmark_graph(const float *L, int g, int d, int kg, int32_t *nbr, double *d2)
{
    if (g < 1 || d < 1 || kg < 1 || !L || !nbr || !d2)
        return ORACLE_EINVAL;
    int *nb = (int *)malloc(sizeof(int) * (size_t)(kg + 1));
    double *nd = (double *)malloc(sizeof(double) * (size_t)(kg + 1));
    if (!nb || !nd) {
        free(nb); free(nd);
        return ORACLE_ENOMEM;
    }
    for (int u = 0; u < g; ++u) {
        /* the kg + 1 nearest include u itself (distance 0, or tied with an
         * exact duplicate); dropping u leaves the kg nearest others */
        nearest_m(L + (size_t)u * d, L, g, d, kg + 1, nb, nd);
        int o = 0;
        for (int i = 0; i < kg + 1 && o < kg; ++i) {
            if (nb[i] == u)
                continue;
            nbr[(size_t)u * kg + o] = nb[i];
            d2[(size_t)u * kg + o] = nb[i] >= 0 ? nd[i] : INFINITY;
            ++o;
        }
        for (; o < kg; ++o) {
            nbr[(size_t)u * kg + o] = -1;
            d2[(size_t)u * kg + o] = INFINITY;
        }
    }
    free(nb); free(nd);
    return ORACLE_OK;
}

/* One synchronous step of the force-based layout of the 2-D landmark
 * positions l (g x 2 floats, updated in place).  Edges: u-v when v is among
 * u's neighbours or u among v's (nbr from oracle_landmark_graph, g x kg), each
 * undirected edge acting once on both ends.  The force on a node u is
 *   sum over edges u-v of (|l_v - l_u| - scale * |L_u - L_v|) (l_v - l_u) / |l_v - l_u|
 *     (a spring whose rest length is the high-dimensional distance times
 *     scale; skipped while the two positions coincide)
 *   + repulsion * sum over all v != u of (l_u - l_v) / (|l_u - l_v|^2 + soft^2).
 * Every node moves by step times its force, shortened to max_move when
 * longer; fixed[u] != 0 (dragged by the user) keeps u in place.  Forces use
 * the positions before the step; sums in double, positions rounded to float. */
int oracle_layout_step(const float *L, int g, int d, const int32_t *nbr, int kg, float *l,
                       const uint8_t *fixed, double scale, double repulsion, double soft,
                       double step, double max_move)
{
    if (g < 1 || d < 1 || kg < 1 || !L || !nbr || !l)
        return ORACLE_EINVAL;
    unsigned char *adj = (unsigned char *)calloc((size_t)g * g, 1);
    double *nl = (double *)malloc(sizeof(double) * 2 * (size_t)g);
    if (!adj || !nl) {
        free(adj); free(nl);
        return ORACLE_ENOMEM;
    }
    for (int u = 0; u < g; ++u)
        for (int i = 0; i < kg; ++i) {
            int v = nbr[(size_t)u * kg + i];
            if (v >= 0 && v != u) {
                adj[(size_t)u * g + v] = 1;
                adj[(size_t)v * g + u] = 1;
            }
        }
    for (int u = 0; u < g; ++u) {
        double ux = l[2 * u], uy = l[2 * u + 1];
        double fx = 0.0, fy = 0.0;
        for (int v = 0; v < g; ++v) {
            if (v == u)
                continue;
            double dx = (double)l[2 * v] - ux, dy = (double)l[2 * v + 1] - uy;
            double r2 = dx * dx + dy * dy;
            if (adj[(size_t)u * g + v]) {
                double r = sqrt(r2);
                if (r > 0.0) {
                    double rest = scale * sqrt(sqdist(L + (size_t)u * d, L + (size_t)v * d, d));
                    fx += (r - rest) * dx / r;
                    fy += (r - rest) * dy / r;
                }
            }
            fx -= repulsion * dx / (r2 + soft * soft);
            fy -= repulsion * dy / (r2 + soft * soft);
        }
        double mx = step * fx, my = step * fy;
        double len = sqrt(mx * mx + my * my);
        if (len > max_move) {
            mx *= max_move / len;
            my *= max_move / len;
        }
        if (fixed && fixed[u])
            mx = my = 0.0;
        nl[2 * u] = ux + mx;
        nl[2 * u + 1] = uy + my;
    }
    for (int e = 0; e < 2 * g; ++e)
        l[e] = (float)nl[e];
    free(adj); free(nl);
    return ORACLE_OK;
}
