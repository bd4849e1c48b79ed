/*
 * gca_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU oracle for the Galerkin matrix of the Laplace
 * single-layer operator with piecewise-constant basis functions on flat
 * triangles:
 *
 *     g_ij = int_{t_i} int_{t_j} g(x,y) dy dx,   g(x,y) = 1 / (4 pi |x - y|)
 *
 * (Section 1: the fundamental solution and Eq. G_def, with phi_i the indicator
 * function of triangle t_i; Section 2 fixes one basis function per triangle.)
 *
 * Only the test-suite, the smoke check and the bench's CPU-baseline leg may
 * load this library.  It shares no code with the HIP library.
 *
 * Quadrature (Section 8: one rule per Sauter case -- identical triangles,
 * common edge, common vertex, disjoint -- citing Sauter and Sauter-Schwab):
 *   - the case is decided combinatorially from vertex indices;
 *   - disjoint pairs use a tensor Gauss rule on each triangle (order q_r, or
 *     q_nr for "near-regular" pairs whose triangles contain two vertices
 *     joined by a mesh edge);
 *   - touching pairs use the regularising 4D transformations on [0,1]^4 of
 *     the Sauter-Schwab method (6 / 5 / 2 subregions) with a q_s-point Gauss
 *     rule in every one of the four variables.
 *
 * Reference triangle:  T = { (s1,s2) : 0 <= s2 <= s1 <= 1 },
 * parametrisation      chi(s) = P0 + s1 (P1 - P0) + s2 (P2 - P1),
 * surface element      |(P1 - P0) x (P2 - P1)| = 2 |t|.
 * Collapsed Gauss rule on T of order q: s1 = u_a, s2 = u_a v_b with weight
 * w_a w_b u_a (u, v, w: Gauss-Legendre on [0,1]).  Optional family for the
 * regular classes ("sym"): the fully symmetric triangle rules of polynomial
 * degree 2q - 2, the same degree as the collapsed rule of order q -- 3 points
 * (degree 2, q = 2) and 6 points (degree 4, q = 3; Strang-Fix / Dunavant),
 * given by barycentric orbits (l0, l1, l2) with s1 = l1 + l2, s2 = l2 and
 * weight w / 2 on T (the weights w sum to one).
 *
 * Vertex order for touching pairs (so that shared vertices come first):
 *   identical  : the mesh order (v0, v1, v2) for both copies;
 *   common edge: shared vertices (a, b) with a < b by vertex id, then the
 *                third vertex of each triangle;
 *   common vertex: the shared vertex, then the other two in cyclic mesh order.
 * Touching and regular values are computed for (min(i,j), max(i,j)) so the
 * matrix is symmetric by construction.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

enum { ORC_REG = 0, ORC_NEAR = 1, ORC_VERT = 2, ORC_EDGE = 3, ORC_IDENT = 4 };

#define ORC_QMAX 32
#define ORC_TMAX (ORC_QMAX * ORC_QMAX)

/* A rule on the reference triangle T: points (s1, s2), weights summing to |T| = 1/2. */
typedef struct {
    int np;
    double s1[ORC_TMAX], s2[ORC_TMAX], w[ORC_TMAX];
} orc_trirule;

typedef struct {
    int64_t nv, nt;
    double *xyz;     /* nv x 3 */
    int32_t *tri;    /* nt x 3 */
    int64_t *vadj_ptr; /* vertex -> neighbouring vertices (mesh edges), CSR */
    int32_t *vadj;
    int q_r, q_nr, q_s, sym;
    orc_trirule rr, rn;                      /* the regular and near-regular triangle rules */
    double gs_x[ORC_QMAX], gs_w[ORC_QMAX];   /* order q_s */
} orc_ctx;

/* Gauss-Legendre rule on [0,1]: nodes are the roots t of the Legendre
 * polynomial P_q on [-1,1], found by Newton's method with P_q and P_q'
 * from the three-term recurrence; x = (1 + t)/2 and w = 1/((1 - t^2) P_q'(t)^2)
 * (the usual weight 2/((1 - t^2) P_q'(t)^2) halved for the interval length).
 * Nodes are returned in ascending order. */
static void legendre_eval(int q, double t, double *p, double *dp)
{
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    /* P_q' from (t^2 - 1) P_q' = q (t P_q - P_{q-1}) */
    *p = p1;
    *dp = q * (t * p1 - p0) / (t * t - 1.0);
}

void orc_gauss01(int q, double *x, double *w)
{
    for (int i = 0; i < q; ++i) {
        /* initial guess for the i-th largest root */
        double t = cos(ORC_PI * (i + 0.75) / (q + 0.5));
        double p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_eval(q, t, &p, &dp);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) <= 1e-16 * fabs(t) + 1e-300) break;
        }
        legendre_eval(q, t, &p, &dp);
        x[q - 1 - i] = 0.5 * (1.0 + t);
        w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);
    }
}

/* Number of OpenMP threads the parallel loops use. */
int orc_num_threads(void) { return omp_get_max_threads(); }

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_destroy(void *p)
{
    orc_ctx *c = (orc_ctx *)p;
    if (!c) return;
    free(c->xyz); free(c->tri); free(c->vadj_ptr); free(c->vadj);
    free(c);
}

/* Collapsed Gauss rule of order q on T (see the header). */
static void rule_collapsed(int q, orc_trirule *r)
{
    double x[ORC_QMAX], w[ORC_QMAX];
    orc_gauss01(q, x, w);
    r->np = 0;
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b) {
            r->s1[r->np] = x[a];
            r->s2[r->np] = x[a] * x[b];
            r->w[r->np] = w[a] * w[b] * x[a];
            r->np++;
        }
}

/* Fully symmetric rule from barycentric orbits: every orbit (a, a, 1 - 2a)
 * contributes its three permutations with barycentric weight w each. */
static void add_orbit(orc_trirule *r, double a, double w)
{
    const double b = 1.0 - 2.0 * a;
    const double l[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
    for (int k = 0; k < 3; ++k) {
        r->s1[r->np] = l[k][1] + l[k][2];
        r->s2[r->np] = l[k][2];
        r->w[r->np] = 0.5 * w;
        r->np++;
    }
}

/* Symmetric rule of degree 2q - 2: q = 2 -> 3 points (orbit a = 1/6, weights
 * 1/3, degree 2); q = 3 -> 6 points (orbits a = 0.445948490915965 with weight
 * 0.223381589678011 and a = 0.091576213509771 with weight 0.109951743655322,
 * degree 4).  Returns 0 for other orders. */
static int rule_symmetric(int q, orc_trirule *r)
{
    r->np = 0;
    if (q == 2) {
        add_orbit(r, 1.0 / 6.0, 1.0 / 3.0);
        return 1;
    }
    if (q == 3) {
        add_orbit(r, 0.445948490915965, 0.223381589678011);
        add_orbit(r, 0.091576213509771, 0.109951743655322);
        return 1;
    }
    return 0;
}

/* The triangle rule the regular classes use (for tests): writes np points
 * (s1, s2) and weights, returns np, or 0 for an unsupported order. */
int orc_tri_rule(int q, int sym, double *s1, double *s2, double *w)
{
    orc_trirule r;
    if (q < 1 || q > ORC_QMAX) return 0;
    if (sym) {
        if (!rule_symmetric(q, &r)) return 0;
    } else {
        rule_collapsed(q, &r);
    }
    for (int k = 0; k < r.np; ++k) { s1[k] = r.s1[k]; s2[k] = r.s2[k]; w[k] = r.w[k]; }
    return r.np;
}

void *orc_create(int64_t nv, int64_t nt, const double *xyz, const int32_t *tri,
                 int q_r, int q_nr, int q_s, int sym)
{
    if (q_r < 1 || q_nr < 1 || q_s < 1 || q_r > ORC_QMAX || q_nr > ORC_QMAX || q_s > ORC_QMAX)
        return NULL;
    if (sym && ((q_r != 2 && q_r != 3) || (q_nr != 2 && q_nr != 3))) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->sym = sym;
    if (sym) {
        rule_symmetric(q_r, &c->rr);
        rule_symmetric(q_nr, &c->rn);
    } else {
        rule_collapsed(q_r, &c->rr);
        rule_collapsed(q_nr, &c->rn);
    }
    c->nv = nv; c->nt = nt;
    c->xyz = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    c->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)nt);
    memcpy(c->xyz, xyz, sizeof(double) * 3 * (size_t)nv);
    memcpy(c->tri, tri, sizeof(int32_t) * 3 * (size_t)nt);
    c->q_r = q_r; c->q_nr = q_nr; c->q_s = q_s;
    orc_gauss01(q_s, c->gs_x, c->gs_w);

    /* vertex adjacency through mesh edges: every triangle contributes its 3 edges
     * in both directions; duplicates removed after sorting */
    int64_t *cnt = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) cnt[tri[3 * t + k] + 1] += 2;
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)cnt[nv]);
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nv);
    for (int64_t v = 0; v < nv; ++v) fill[v] = cnt[v];
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3], d = tri[3 * t + (k + 2) % 3];
            tmp[fill[a]++] = b;
            tmp[fill[a]++] = d;
        }
    c->vadj_ptr = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    c->vadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[nv] > 0 ? cnt[nv] : 1));
    int64_t o = 0;
    for (int64_t v = 0; v < nv; ++v) {
        int64_t b = cnt[v], e = cnt[v + 1];
        qsort(tmp + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        c->vadj_ptr[v] = o;
        for (int64_t k = b; k < e; ++k)
            if (k == b || tmp[k] != tmp[k - 1]) c->vadj[o++] = tmp[k];
    }
    c->vadj_ptr[nv] = o;
    free(cnt); free(tmp); free(fill);
    return c;
}

static int is_edge(const orc_ctx *c, int32_t a, int32_t b)
{
    for (int64_t k = c->vadj_ptr[a]; k < c->vadj_ptr[a + 1]; ++k)
        if (c->vadj[k] == b) return 1;
    return 0;
}

/* Pair class decided from vertex indices only. */
int orc_classify(void *p, int64_t i, int64_t j)
{
    const orc_ctx *c = (const orc_ctx *)p;
    const int32_t *ti = c->tri + 3 * i, *tj = c->tri + 3 * j;
    int shared = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ti[a] == tj[b]) ++shared;
    if (shared == 3) return ORC_IDENT;
    if (shared == 2) return ORC_EDGE;
    if (shared == 1) return ORC_VERT;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (is_edge(c, ti[a], tj[b])) return ORC_NEAR;
    return ORC_REG;
}

static void vload(const orc_ctx *c, int32_t v, double *out)
{
    out[0] = c->xyz[3 * v]; out[1] = c->xyz[3 * v + 1]; out[2] = c->xyz[3 * v + 2];
}

/* chi(s) - P0 = s1 (P1 - P0) + s2 (P2 - P1) for a triangle given by vertices P */
static void chi_rel(const double P[3][3], double s1, double s2, double *out)
{
    for (int d = 0; d < 3; ++d)
        out[d] = s1 * (P[1][d] - P[0][d]) + s2 * (P[2][d] - P[1][d]);
}

static double surf_elem(const double P[3][3])
{
    double a[3], b[3];
    for (int d = 0; d < 3; ++d) { a[d] = P[1][d] - P[0][d]; b[d] = P[2][d] - P[1][d]; }
    double cx = a[1] * b[2] - a[2] * b[1];
    double cy = a[2] * b[0] - a[0] * b[2];
    double cz = a[0] * b[1] - a[1] * b[0];
    return sqrt(cx * cx + cy * cy + cz * cz);
}

/* Regular rule: the triangle rule r on both triangles. */
static double entry_regular(const double P[3][3], const double Q[3][3], const orc_trirule *r)
{
    double Jp = surf_elem(P), Jq = surf_elem(Q);
    double sum = 0.0;
    for (int a = 0; a < r->np; ++a) {
        double x[3];
        chi_rel(P, r->s1[a], r->s2[a], x);
        for (int d = 0; d < 3; ++d) x[d] += P[0][d];
        for (int b = 0; b < r->np; ++b) {
            double y[3];
            chi_rel(Q, r->s1[b], r->s2[b], y);
            for (int d = 0; d < 3; ++d) y[d] += Q[0][d];
            double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
            sum += r->w[a] * r->w[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    return sum * Jp * Jq / (4.0 * ORC_PI);
}

/* Sauter-Schwab regularising maps of [0,1]^4 onto T x T for the three touching
 * cases.  Returns the Jacobian; (x1,x2) in the first, (y1,y2) in the second
 * triangle's reference coordinates.  The singular set (x = y, the shared edge
 * x2 = y2 = 0, x1 = y1, or the shared vertex x = y = 0) is mapped to the faces
 * xi = 0 / eta1 = 0 where the Jacobian vanishes to the order that cancels the
 * 1/|x - y| singularity. */
static double ss_map(int kase, int region, double xi, double e1, double e2, double e3,
                     double *x1, double *x2, double *y1, double *y2)
{
    if (kase == ORC_IDENT) {
        double J = xi * xi * xi * e1 * e1 * e2;
        switch (region) {
        case 0: *x1 = xi; *x2 = xi * (1 - e1 + e1 * e2); *y1 = xi * (1 - e1 * e2 * e3); *y2 = xi * (1 - e1); break;
        case 1: *x1 = xi * (1 - e1 * e2 * e3); *x2 = xi * (1 - e1); *y1 = xi; *y2 = xi * (1 - e1 + e1 * e2); break;
        case 2: *x1 = xi; *x2 = xi * e1 * (1 - e2 + e2 * e3); *y1 = xi * (1 - e1 * e2); *y2 = xi * e1 * (1 - e2); break;
        case 3: *x1 = xi * (1 - e1 * e2); *x2 = xi * e1 * (1 - e2); *y1 = xi; *y2 = xi * e1 * (1 - e2 + e2 * e3); break;
        case 4: *x1 = xi * (1 - e1 * e2 * e3); *x2 = xi * e1 * (1 - e2 * e3); *y1 = xi; *y2 = xi * e1 * (1 - e2); break;
        default: *x1 = xi; *x2 = xi * e1 * (1 - e2); *y1 = xi * (1 - e1 * e2 * e3); *y2 = xi * e1 * (1 - e2 * e3); break;
        }
        return J;
    }
    if (kase == ORC_EDGE) {
        switch (region) {
        case 0: *x1 = xi; *x2 = xi * e1 * e3; *y1 = xi * (1 - e1 * e2); *y2 = xi * e1 * (1 - e2);
            return xi * xi * xi * e1 * e1;
        case 1: *x1 = xi; *x2 = xi * e1; *y1 = xi * (1 - e1 * e2 * e3); *y2 = xi * e1 * e2 * (1 - e3); break;
        case 2: *x1 = xi * (1 - e1 * e2); *x2 = xi * e1 * (1 - e2); *y1 = xi; *y2 = xi * e1 * e2 * e3; break;
        case 3: *x1 = xi * (1 - e1 * e2 * e3); *x2 = xi * e1 * e2 * (1 - e3); *y1 = xi; *y2 = xi * e1; break;
        default: *x1 = xi * (1 - e1 * e2 * e3); *x2 = xi * e1 * (1 - e2 * e3); *y1 = xi; *y2 = xi * e1 * e2; break;
        }
        return xi * xi * xi * e1 * e1 * e2;
    }
    /* common vertex */
    if (region == 0) { *x1 = xi; *x2 = xi * e1; *y1 = xi * e2; *y2 = xi * e2 * e3; }
    else             { *x1 = xi * e2; *x2 = xi * e2 * e3; *y1 = xi; *y2 = xi * e1; }
    return xi * xi * xi * e2;
}

static int ss_regions(int kase) { return kase == ORC_IDENT ? 6 : (kase == ORC_EDGE ? 5 : 2); }

/* Integral over T x T of a function of the two reference points, by the
 * Sauter-Schwab maps with a q-point Gauss rule in each of the four variables.
 * P and Q share their first vertex (edge case: first two), so
 * chi_P(x) - chi_Q(y) = (chi_P(x) - P0) - (chi_Q(y) - Q0). */
static double entry_touching(int kase, const double P[3][3], const double Q[3][3],
                             int q, const double *gx, const double *gw)
{
    double Jp = surf_elem(P), Jq = surf_elem(Q);
    int nreg = ss_regions(kase);
    double sum = 0.0;
    for (int r = 0; r < nreg; ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, gx[a], gx[b], gx[e], gx[f], &x1, &x2, &y1, &y2);
                        double w = gw[a] * gw[b] * gw[e] * gw[f] * jac;
                        double X[3], Y[3];
                        chi_rel(P, x1, x2, X);
                        chi_rel(Q, y1, y2, Y);
                        double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                        sum += w / sqrt(dx * dx + dy * dy + dz * dz);
                    }
    return sum * Jp * Jq / (4.0 * ORC_PI);
}

/* Moments of the Sauter-Schwab maps: sum of weights times x1^a x2^b y1^c y2^d.
 * Equals int_T int_T x1^a x2^b y1^c y2^d exactly when the maps tile T x T. */
double orc_ss_moment(int kase, int q, int pa, int pb, int pc, int pd)
{
    double gx[ORC_QMAX], gw[ORC_QMAX];
    if (q < 1 || q > ORC_QMAX) return NAN;
    orc_gauss01(q, gx, gw);
    double sum = 0.0;
    for (int r = 0; r < ss_regions(kase); ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, gx[a], gx[b], gx[e], gx[f], &x1, &x2, &y1, &y2);
                        sum += gw[a] * gw[b] * gw[e] * gw[f] * jac *
                               pow(x1, pa) * pow(x2, pb) * pow(y1, pc) * pow(y2, pd);
                    }
    return sum;
}

/* Orders the vertices of the pair (i, j), i <= j, for the touching rules. */
static void touching_vertices(const orc_ctx *c, int kase, int64_t i, int64_t j,
                              double P[3][3], double Q[3][3], int32_t *pid, int32_t *qid)
{
    const int32_t *ti = c->tri + 3 * i, *tj = c->tri + 3 * j;
    int32_t pi[3], pj[3];
    if (kase == ORC_IDENT) {
        for (int k = 0; k < 3; ++k) { pi[k] = ti[k]; pj[k] = ti[k]; }
    } else if (kase == ORC_EDGE) {
        int32_t sh[2]; int ns = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (ti[a] == tj[b]) sh[ns++] = ti[a];
        int32_t lo = sh[0] < sh[1] ? sh[0] : sh[1];
        int32_t hi = sh[0] < sh[1] ? sh[1] : sh[0];
        int32_t oi = -1, oj = -1;
        for (int a = 0; a < 3; ++a) if (ti[a] != lo && ti[a] != hi) oi = ti[a];
        for (int b = 0; b < 3; ++b) if (tj[b] != lo && tj[b] != hi) oj = tj[b];
        pi[0] = lo; pi[1] = hi; pi[2] = oi;
        pj[0] = lo; pj[1] = hi; pj[2] = oj;
    } else {
        int ka = 0, kb = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (ti[a] == tj[b]) { ka = a; kb = b; }
        for (int k = 0; k < 3; ++k) { pi[k] = ti[(ka + k) % 3]; pj[k] = tj[(kb + k) % 3]; }
    }
    for (int k = 0; k < 3; ++k) { vload(c, pi[k], P[k]); vload(c, pj[k], Q[k]); }
    if (pid) for (int k = 0; k < 3; ++k) { pid[k] = pi[k]; qid[k] = pj[k]; }
}

double orc_entry(void *p, int64_t i, int64_t j)
{
    const orc_ctx *c = (const orc_ctx *)p;
    if (i > j) { int64_t t = i; i = j; j = t; }
    int kase = orc_classify(p, i, j);
    double P[3][3], Q[3][3];
    if (kase == ORC_IDENT || kase == ORC_EDGE || kase == ORC_VERT) {
        touching_vertices(c, kase, i, j, P, Q, NULL, NULL);
        return entry_touching(kase, P, Q, c->q_s, c->gs_x, c->gs_w);
    }
    for (int k = 0; k < 3; ++k) { vload(c, c->tri[3 * i + k], P[k]); vload(c, c->tri[3 * j + k], Q[k]); }
    if (kase == ORC_NEAR) return entry_regular(P, Q, &c->rn);
    return entry_regular(P, Q, &c->rr);
}

void orc_entries(void *p, int64_t m, const int64_t *I, const int64_t *J, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < m; ++k) out[k] = orc_entry(p, I[k], J[k]);
}

void orc_classify_many(void *p, int64_t m, const int64_t *I, const int64_t *J, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) out[k] = orc_classify(p, I[k], J[k]);
}

/* Dense G, row-major n x n (upper triangle computed, mirrored). */
void orc_dense(void *p, double *G)
{
    const orc_ctx *c = (const orc_ctx *)p;
    int64_t n = c->nt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            double v = orc_entry(p, i, j);
            G[i * n + j] = v;
            G[j * n + i] = v;
        }
}

/* y[r, :] = sum_j g_{rows[r], j} x[j, :] for the requested rows, without storing G.
 * x is n x nrhs row-major, y is nrows x nrhs row-major. */
void orc_matvec_rows(void *p, int64_t nrows, const int64_t *rows, const double *x,
                     int64_t nrhs, double *y)
{
    const orc_ctx *c = (const orc_ctx *)p;
    int64_t n = c->nt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        double *yr = y + r * nrhs;
        for (int64_t k = 0; k < nrhs; ++k) yr[k] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double g = orc_entry(p, rows[r], j);
            for (int64_t k = 0; k < nrhs; ++k) yr[k] += g * x[j * nrhs + k];
        }
    }
}

/* Triangle quadrature points of the collapsed rule of order q (for the
 * Green-quadrature factor entries): pts (nt*q*q x 3), weights incl. surface
 * element (nt*q*q). */
void orc_triangle_points(void *p, int q, double *pts, double *wts)
{
    const orc_ctx *c = (const orc_ctx *)p;
    double gx[ORC_QMAX], gw[ORC_QMAX];
    orc_gauss01(q, gx, gw);
    for (int64_t t = 0; t < c->nt; ++t) {
        double P[3][3];
        for (int k = 0; k < 3; ++k) vload(c, c->tri[3 * t + k], P[k]);
        double J = surf_elem(P);
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                int64_t o = (t * q + a) * q + b;
                double x[3];
                chi_rel(P, gx[a], gx[a] * gx[b], x);
                for (int d = 0; d < 3; ++d) pts[3 * o + d] = x[d] + P[0][d];
                wts[o] = gw[a] * gw[b] * gx[a] * J;
            }
    }
}

/* ------------------------------------------------------------------------
 * Derivatives of the entries with respect to the vertex coordinates (for the
 * energy E = 1/2 u^T G u and the adjoint of the H^2 product).
 *
 * Every rule above integrates F = w J_P J_Q / (4 pi |X - Y|) at fixed
 * reference points, with X = b0 P0 + b1 P1 + b2 P2, (b0, b1, b2) =
 * (1 - s1, s1 - s2, s2), J = |(P1 - P0) x (P2 - P1)|.  The derivative of F with
 * respect to a vertex copy P_k is therefore
 *     w [ dJ_P/dP_k J_Q / r - J_P J_Q (X - Y) b_k / r^3 ] / (4 pi),
 * and likewise for Q_k with the opposite sign of the second term.  Shared
 * vertices appear once in each triangle; their two partial derivatives add.
 * ------------------------------------------------------------------------ */

/* dJ/dP_k for J = |(P1 - P0) x (P2 - P1)|: with e1 = P1 - P0, e2 = P2 - P1,
 * c = e1 x e2, dJ/de1 = e2 x c/|c|, dJ/de2 = c/|c| x e1. */
static void surf_elem_grad(const double P[3][3], double g[3][3])
{
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[1][d]; }
    double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double J = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int d = 0; d < 3; ++d) c[d] /= J;
    double a[3] = {e2[1] * c[2] - e2[2] * c[1], e2[2] * c[0] - e2[0] * c[2], e2[0] * c[1] - e2[1] * c[0]};  /* dJ/de1 */
    double b[3] = {c[1] * e1[2] - c[2] * e1[1], c[2] * e1[0] - c[0] * e1[2], c[0] * e1[1] - c[1] * e1[0]};  /* dJ/de2 */
    for (int d = 0; d < 3; ++d) {
        g[0][d] = -a[d];
        g[1][d] = a[d] - b[d];
        g[2][d] = b[d];
    }
}

/* One quadrature point pair: adds to GP (d/dP_k) and GQ (d/dQ_k). */
static void grad_point(const double P[3][3], const double Q[3][3], double JP, double JQ,
                       const double gJP[3][3], const double gJQ[3][3],
                       double s1, double s2, double u1, double u2, double w,
                       const double *XmY, double GP[3][3], double GQ[3][3])
{
    double r2 = XmY[0] * XmY[0] + XmY[1] * XmY[1] + XmY[2] * XmY[2];
    double r = sqrt(r2);
    double bp[3] = {1.0 - s1, s1 - s2, s2}, bq[3] = {1.0 - u1, u1 - u2, u2};
    double f = w / r, h = w * JP * JQ / (r2 * r);
    (void)P; (void)Q;
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
            GP[k][d] += f * gJP[k][d] * JQ - h * XmY[d] * bp[k];
            GQ[k][d] += f * JP * gJQ[k][d] + h * XmY[d] * bq[k];
        }
}

static void grad_regular(const double P[3][3], const double Q[3][3], const orc_trirule *r, double GP[3][3],
                         double GQ[3][3])
{
    double JP = surf_elem(P), JQ = surf_elem(Q);
    double gJP[3][3], gJQ[3][3];
    surf_elem_grad(P, gJP);
    surf_elem_grad(Q, gJQ);
    for (int a = 0; a < r->np; ++a) {
        const double s1 = r->s1[a], s2 = r->s2[a];
        double x[3];
        chi_rel(P, s1, s2, x);
        for (int d = 0; d < 3; ++d) x[d] += P[0][d];
        for (int b = 0; b < r->np; ++b) {
            const double u1 = r->s1[b], u2 = r->s2[b];
            double y[3], XmY[3];
            chi_rel(Q, u1, u2, y);
            for (int d = 0; d < 3; ++d) XmY[d] = x[d] - (y[d] + Q[0][d]);
            grad_point(P, Q, JP, JQ, gJP, gJQ, s1, s2, u1, u2, r->w[a] * r->w[b], XmY, GP, GQ);
        }
    }
}

static void grad_touching(int kase, const double P[3][3], const double Q[3][3], int q, const double *gx,
                          const double *gw, double GP[3][3], double GQ[3][3])
{
    double JP = surf_elem(P), JQ = surf_elem(Q);
    double gJP[3][3], gJQ[3][3];
    surf_elem_grad(P, gJP);
    surf_elem_grad(Q, gJQ);
    int nreg = ss_regions(kase);
    for (int r = 0; r < nreg; ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, gx[a], gx[b], gx[e], gx[f], &x1, &x2, &y1, &y2);
                        double w = gw[a] * gw[b] * gw[e] * gw[f] * jac;
                        double X[3], Y[3], XmY[3];
                        chi_rel(P, x1, x2, X);
                        chi_rel(Q, y1, y2, Y);
                        /* P0 and Q0 are the same vertex: X - Y = (P0 - Q0) + ... = rel. parts */
                        for (int d = 0; d < 3; ++d) XmY[d] = (P[0][d] - Q[0][d]) + X[d] - Y[d];
                        grad_point(P, Q, JP, JQ, gJP, gJQ, x1, x2, y1, y2, w, XmY, GP, GQ);
                    }
}

/* local slot of vertex id v in triangle t */
static int local_slot(const orc_ctx *c, int64_t t, int32_t v)
{
    for (int k = 0; k < 3; ++k)
        if (c->tri[3 * t + k] == v) return k;
    return -1;
}

/* out[0..8]: d g_ij / d(vertex slot m of t_i, coordinate d) at 3 m + d;
 * out[9..17]: the same for t_j.  For i == j the whole derivative of g_ii is in
 * out[0..8] and out[9..17] is zero. */
void orc_entry_grad(void *p, int64_t i, int64_t j, double *out)
{
    const orc_ctx *c = (const orc_ctx *)p;
    for (int k = 0; k < 18; ++k) out[k] = 0.0;
    int swapped = 0;
    if (i > j) { int64_t t = i; i = j; j = t; swapped = 1; }
    int kase = orc_classify(p, i, j);
    double P[3][3], Q[3][3], GP[3][3] = {{0}}, GQ[3][3] = {{0}};
    int32_t pid[3], qid[3];
    if (kase == ORC_IDENT || kase == ORC_EDGE || kase == ORC_VERT) {
        touching_vertices(c, kase, i, j, P, Q, pid, qid);
        grad_touching(kase, P, Q, c->q_s, c->gs_x, c->gs_w, GP, GQ);
    } else {
        for (int k = 0; k < 3; ++k) {
            pid[k] = c->tri[3 * i + k];
            qid[k] = c->tri[3 * j + k];
            vload(c, pid[k], P[k]);
            vload(c, qid[k], Q[k]);
        }
        if (kase == ORC_NEAR) grad_regular(P, Q, &c->rn, GP, GQ);
        else grad_regular(P, Q, &c->rr, GP, GQ);
    }
    double *oi = out + (swapped ? 9 : 0), *oj = out + (swapped ? 0 : 9);
    if (i == j) { oi = out; oj = out; }
    for (int k = 0; k < 3; ++k) {
        int si = local_slot(c, i, pid[k]), sj = local_slot(c, j, qid[k]);
        for (int d = 0; d < 3; ++d) {
            oi[3 * si + d] += GP[k][d] / (4.0 * ORC_PI);
            oj[3 * sj + d] += GQ[k][d] / (4.0 * ORC_PI);
        }
    }
}

/* dE/dX for E = 1/2 u^T G u at the selected vertices (nsel x 3, row-major):
 * dE/dX_v = sum over triangles t containing v of u_t sum_j u_j d_t g_tj (the
 * t-side partial derivative; the identical pair contributes half of its full
 * derivative, as both copies of t lie in t). */
void orc_energy_grad_vertices(void *p, const double *u, int64_t nsel, const int32_t *vsel, double *out)
{
    const orc_ctx *c = (const orc_ctx *)p;
    const int64_t n = c->nt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsel; ++s) {
        const int32_t v = vsel[s];
        double acc[3] = {0, 0, 0};
        for (int64_t t = 0; t < n; ++t) {
            int slot = local_slot(c, t, v);
            if (slot < 0) continue;
            for (int64_t j = 0; j < n; ++j) {
                double g[18];
                orc_entry_grad(p, t, j, g);
                double wgt = u[t] * u[j] * (j == t ? 0.5 : 1.0);
                for (int d = 0; d < 3; ++d) acc[d] += wgt * g[3 * slot + d];
            }
        }
        for (int d = 0; d < 3; ++d) out[3 * s + d] = acc[d];
    }
}

/* ------------------------------------------------------------------------
 * Double-layer kernel (Section 1: the second-kind formulation uses the normal
 * derivative of g at y; Section 6: unit normals of the triangles):
 *     k_ij = int_{t_i} int_{t_j} dg/dn_y(x, y) dy dx,
 *     dg/dn_y(x, y) = n_j . (x - y) / (4 pi |x - y|^3),
 * n_j the unit normal of t_j from its mesh orientation (v1 - v0) x (v2 - v0).
 * Not symmetric: x runs over t_i, y over t_j.  Identical pairs are 0 (the
 * two points lie in one plane, n_j . (x - y) = 0); touching pairs use the
 * same Sauter-Schwab maps as above (the kernel is O(1/r^2) near the common
 * edge or vertex, which the Jacobian's xi^3 cancels), the others the regular
 * rules of the single-layer entries. */

static void unit_normal(const orc_ctx *c, int64_t t, double *n)
{
    double P[3][3];
    for (int k = 0; k < 3; ++k) vload(c, c->tri[3 * t + k], P[k]);
    double a[3], b[3];
    for (int d = 0; d < 3; ++d) { a[d] = P[1][d] - P[0][d]; b[d] = P[2][d] - P[0][d]; }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int d = 0; d < 3; ++d) n[d] /= l;
}

static double entry_regular_dl(const double P[3][3], const double Q[3][3], const double *n, const orc_trirule *r)
{
    double Jp = surf_elem(P), Jq = surf_elem(Q);
    double sum = 0.0;
    for (int a = 0; a < r->np; ++a) {
        double x[3];
        chi_rel(P, r->s1[a], r->s2[a], x);
        for (int d = 0; d < 3; ++d) x[d] += P[0][d];
        for (int b = 0; b < r->np; ++b) {
            double y[3];
            chi_rel(Q, r->s1[b], r->s2[b], y);
            for (int d = 0; d < 3; ++d) y[d] += Q[0][d];
            double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
            double r2 = dx * dx + dy * dy + dz * dz;
            sum += r->w[a] * r->w[b] * (n[0] * dx + n[1] * dy + n[2] * dz) / (r2 * sqrt(r2));
        }
    }
    return sum * Jp * Jq / (4.0 * ORC_PI);
}

static double entry_touching_dl(int kase, const double P[3][3], const double Q[3][3], const double *n,
                                int q, const double *gx, const double *gw)
{
    double Jp = surf_elem(P), Jq = surf_elem(Q);
    int nreg = ss_regions(kase);
    double sum = 0.0;
    for (int r = 0; r < nreg; ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, gx[a], gx[b], gx[e], gx[f], &x1, &x2, &y1, &y2);
                        double w = gw[a] * gw[b] * gw[e] * gw[f] * jac;
                        double X[3], Y[3];
                        chi_rel(P, x1, x2, X);
                        chi_rel(Q, y1, y2, Y);
                        double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                        double r2 = dx * dx + dy * dy + dz * dz;
                        sum += w * (n[0] * dx + n[1] * dy + n[2] * dz) / (r2 * sqrt(r2));
                    }
    return sum * Jp * Jq / (4.0 * ORC_PI);
}

double orc_entry_dl(void *p, int64_t i, int64_t j)
{
    const orc_ctx *c = (const orc_ctx *)p;
    int kase = orc_classify(p, i < j ? i : j, i < j ? j : i);
    if (kase == ORC_IDENT) return 0.0;
    double n[3];
    unit_normal(c, j, n);
    double P[3][3], Q[3][3];
    if (kase == ORC_EDGE || kase == ORC_VERT) {
        touching_vertices(c, kase, i, j, P, Q, NULL, NULL);
        return entry_touching_dl(kase, P, Q, n, c->q_s, c->gs_x, c->gs_w);
    }
    for (int k = 0; k < 3; ++k) { vload(c, c->tri[3 * i + k], P[k]); vload(c, c->tri[3 * j + k], Q[k]); }
    return entry_regular_dl(P, Q, n, kase == ORC_NEAR ? &c->rn : &c->rr);
}

void orc_entries_dl(void *p, int64_t m, const int64_t *I, const int64_t *J, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < m; ++k) out[k] = orc_entry_dl(p, I[k], J[k]);
}

/* ------------------------------------------------------------------------
 * Continuous piecewise-linear nodal basis (Section 5): the nine corner moments
 * of a touching triangle pair (t, s),
 *     M[a][b] = int_t int_s lambda_a(x) g(x, y) lambda_b(y) dy dx,
 * a, b the corners of t and s in mesh order, by the same Sauter-Schwab maps
 * and q_s-point Gauss rules as the piecewise-constant entries, with the
 * barycentric weights (1 - s1, s1 - s2, s2) of the maps' reference points
 * (in the vertex order of the rule) moved back to mesh order.  Sets NaN for a
 * pair that does not touch. */
void orc_lin_touch_moments(void *p, int64_t t, int64_t s, double *M)
{
    const orc_ctx *c = (const orc_ctx *)p;
    int kase = orc_classify(p, t < s ? t : s, t < s ? s : t);
    for (int k = 0; k < 9; ++k) M[k] = 0.0;
    if (kase != ORC_IDENT && kase != ORC_EDGE && kase != ORC_VERT) {
        for (int k = 0; k < 9; ++k) M[k] = NAN;
        return;
    }
    double P[3][3], Q[3][3];
    int32_t pid[3], qid[3];
    touching_vertices(c, kase, t, s, P, Q, pid, qid);
    int ca[3], cb[3];
    for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) {
            if (c->tri[3 * t + m] == pid[k]) ca[k] = m;
            if (c->tri[3 * s + m] == qid[k]) cb[k] = m;
        }
    double Jp = surf_elem(P), Jq = surf_elem(Q);
    int q = c->q_s;
    for (int r = 0; r < ss_regions(kase); ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, c->gs_x[a], c->gs_x[b], c->gs_x[e], c->gs_x[f],
                                            &x1, &x2, &y1, &y2);
                        double w = c->gs_w[a] * c->gs_w[b] * c->gs_w[e] * c->gs_w[f] * jac;
                        double X[3], Y[3];
                        chi_rel(P, x1, x2, X);
                        chi_rel(Q, y1, y2, Y);
                        double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                        double g = w / sqrt(dx * dx + dy * dy + dz * dz);
                        double lp[3] = {1.0 - x1, x1 - x2, x2}, lq[3] = {1.0 - y1, y1 - y2, y2};
                        for (int k = 0; k < 3; ++k)
                            for (int m = 0; m < 3; ++m) M[3 * ca[k] + cb[m]] += g * lp[k] * lq[m];
                    }
    for (int k = 0; k < 9; ++k) M[k] *= Jp * Jq / (4.0 * ORC_PI);
}

/* ------------------------------------------------------------------------
 * Curved (quadratic) triangles (Section 6).  Triangle t is the image of the
 * reference triangle under the quadratic map Phi_t that interpolates its
 * vertices X0, X1, X2 and the points X3, X4, X5 given for its edges X0-X1,
 * X1-X2, X2-X0 at the edge midpoints.  With the barycentric coordinates
 * (l0, l1, l2) = (1 - s1, s1 - s2, s2) of the reference point s (the
 * parametrisation of the flat code above, whose map is the special case of
 * straight-edge midpoints):
 *     Phi(s) = sum_a l_a (2 l_a - 1) X_a + 4 l0 l1 X3 + 4 l1 l2 X4 + 4 l2 l0 X5,
 * the normal n(s) = dPhi/ds1 x dPhi/ds2 and the Gramian gamma(s) = |n(s)|.
 * The basis functions are the mapped nodal functions: phi_a o Phi = l_a.
 * For a pair (t, s) the nine moments
 *     M[a][b] = int_that int_that l_a(x) k(Phi_t(x), Phi_s(y)) l_b(y)
 *               gamma_t(x) gamma_s(y) dy dx
 * are returned (a, b corners in mesh order; the piecewise-constant entry is
 * their sum) for k the single-layer kernel g (op 0) or the double-layer
 * kernel n_s(y) . (x - y) / (4 pi |x - y|^3) with the unit normal
 * n_s = n / gamma of the mesh orientation (op 1).  Touching pairs, decided
 * by the corner ids, use the Sauter-Schwab maps of the flat entries on the
 * reference coordinates, with the corners reordered as there (the edge
 * points follow their edges) and differences Phi_t(x) - Phi_s(y) formed
 * relative to the shared vertex; the others the regular rule on both
 * triangles. */

typedef struct {
    int64_t nn, nt;
    double *xyz;     /* nn x 3 nodes */
    int32_t *tri;    /* nt x 6: X0 X1 X2 (corners) and the edge points of X0-X1, X1-X2, X2-X0 */
    int q_s;
    orc_trirule rr;
    double gs_x[ORC_QMAX], gs_w[ORC_QMAX];
} orc_curved;

void *orc_curved_create(int64_t nn, int64_t nt, const double *xyz, const int32_t *tri6, int q_r, int q_s, int sym)
{
    if (q_r < 1 || q_s < 1 || q_r > ORC_QMAX || q_s > ORC_QMAX) return NULL;
    if (sym && q_r != 2 && q_r != 3) return NULL;
    orc_curved *c = (orc_curved *)calloc(1, sizeof(orc_curved));
    if (sym) rule_symmetric(q_r, &c->rr);
    else rule_collapsed(q_r, &c->rr);
    c->nn = nn; c->nt = nt; c->q_s = q_s;
    c->xyz = (double *)malloc(sizeof(double) * 3 * (size_t)nn);
    c->tri = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)nt);
    memcpy(c->xyz, xyz, sizeof(double) * 3 * (size_t)nn);
    memcpy(c->tri, tri6, sizeof(int32_t) * 6 * (size_t)nt);
    orc_gauss01(q_s, c->gs_x, c->gs_w);
    return c;
}

void orc_curved_destroy(void *p)
{
    orc_curved *c = (orc_curved *)p;
    if (!c) return;
    free(c->xyz); free(c->tri); free(c);
}

/* ORC_IDENT / ORC_EDGE / ORC_VERT by shared corners, else ORC_REG */
int orc_curved_classify(void *p, int64_t i, int64_t j)
{
    const orc_curved *c = (const orc_curved *)p;
    int shared = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (c->tri[6 * i + a] == c->tri[6 * j + b]) ++shared;
    return shared == 3 ? ORC_IDENT : (shared == 2 ? ORC_EDGE : (shared == 1 ? ORC_VERT : ORC_REG));
}

/* node index (3, 4, 5) of the edge between corners a and b */
static int edge_slot(int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 3 : 5) : 4;
}

/* The six nodes of triangle t with its corners taken in the order perm
 * (new corner k = mesh corner perm[k]). */
static void curved_nodes(const orc_curved *c, int64_t t, const int *perm, double X[6][3])
{
    int src[6] = {perm[0], perm[1], perm[2], edge_slot(perm[0], perm[1]), edge_slot(perm[1], perm[2]),
                  edge_slot(perm[2], perm[0])};
    for (int k = 0; k < 6; ++k)
        for (int d = 0; d < 3; ++d) X[k][d] = c->xyz[3 * (int64_t)c->tri[6 * t + src[k]] + d];
}

/* Phi(s) - X0 and n(s) */
static void curved_eval(const double X[6][3], double s1, double s2, double *rel, double *n)
{
    double l0 = 1.0 - s1, l1 = s1 - s2, l2 = s2;
    double N[6] = {l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), 4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0};
    /* derivatives of the shape functions with respect to (l0, l1, l2) */
    double D[6][3] = {{4 * l0 - 1, 0, 0}, {0, 4 * l1 - 1, 0}, {0, 0, 4 * l2 - 1},
                      {4 * l1, 4 * l0, 0}, {0, 4 * l2, 4 * l1}, {4 * l2, 0, 4 * l0}};
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        rel[d] = 0.0;
        for (int k = 0; k < 6; ++k) {
            rel[d] += N[k] * (X[k][d] - X[0][d]);
            /* d/ds1 = d/dl1 - d/dl0, d/ds2 = d/dl2 - d/dl1 */
            a[d] += (D[k][1] - D[k][0]) * X[k][d];
            b[d] += (D[k][2] - D[k][1]) * X[k][d];
        }
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
}

/* kernel value times gamma_t gamma_s: op 0 g gamma_s, op 1 (ns . d) / (4 pi r^3) with
 * ns = sign * n_s (the unnormalised normal of the mesh orientation) */
static double curved_kernel(int op, const double *d, const double *ns, double sign)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (op == 0) return sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]) / (4.0 * ORC_PI * sqrt(r2));
    return sign * (ns[0] * d[0] + ns[1] * d[1] + ns[2] * d[2]) / (4.0 * ORC_PI * r2 * sqrt(r2));
}

static double vnorm(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* sign of a permutation of (0, 1, 2) */
static double perm_sign(const int *p)
{
    int inv = (p[0] > p[1]) + (p[0] > p[2]) + (p[1] > p[2]);
    return (inv & 1) ? -1.0 : 1.0;
}

void orc_curved_moments(void *p, int op, int64_t t, int64_t s, double *M)
{
    const orc_curved *c = (const orc_curved *)p;
    for (int k = 0; k < 9; ++k) M[k] = 0.0;
    const int32_t *vt = c->tri + 6 * t, *vs = c->tri + 6 * s;
    int kase = orc_curved_classify(p, t, s);
    int pa[3] = {0, 1, 2}, pb[3] = {0, 1, 2};
    if (kase == ORC_EDGE) {
        int sa[2], sb[2], ns = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (vt[a] == vs[b]) { sa[ns] = a; sb[ns] = b; ++ns; }
        int lo0 = vt[sa[0]] < vt[sa[1]];
        pa[0] = lo0 ? sa[0] : sa[1]; pa[1] = lo0 ? sa[1] : sa[0]; pa[2] = 3 - pa[0] - pa[1];
        pb[0] = lo0 ? sb[0] : sb[1]; pb[1] = lo0 ? sb[1] : sb[0]; pb[2] = 3 - pb[0] - pb[1];
    } else if (kase == ORC_VERT) {
        int ka = 0, kb = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (vt[a] == vs[b]) { ka = a; kb = b; }
        for (int k = 0; k < 3; ++k) { pa[k] = (ka + k) % 3; pb[k] = (kb + k) % 3; }
    }
    double X[6][3], Y[6][3];
    curved_nodes(c, t, pa, X);
    curved_nodes(c, s, pb, Y);
    double sgn = perm_sign(pb);
    if (kase == ORC_REG) {
        const orc_trirule *r = &c->rr;
        for (int a = 0; a < r->np; ++a) {
            double xr[3], nx[3];
            curved_eval(X, r->s1[a], r->s2[a], xr, nx);
            double lp[3] = {1.0 - r->s1[a], r->s1[a] - r->s2[a], r->s2[a]};
            double wx = r->w[a] * vnorm(nx);
            for (int b = 0; b < r->np; ++b) {
                double yr[3], ny[3], d[3];
                curved_eval(Y, r->s1[b], r->s2[b], yr, ny);
                for (int k = 0; k < 3; ++k) d[k] = (X[0][k] + xr[k]) - (Y[0][k] + yr[k]);
                double g = wx * r->w[b] * curved_kernel(op, d, ny, sgn);
                double lq[3] = {1.0 - r->s1[b], r->s1[b] - r->s2[b], r->s2[b]};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) M[3 * pa[i] + pb[j]] += g * lp[i] * lq[j];
            }
        }
        return;
    }
    int q = c->q_s;
    for (int r = 0; r < ss_regions(kase); ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int e = 0; e < q; ++e)
                    for (int f = 0; f < q; ++f) {
                        double x1, x2, y1, y2;
                        double jac = ss_map(kase, r, c->gs_x[a], c->gs_x[b], c->gs_x[e], c->gs_x[f], &x1, &x2, &y1, &y2);
                        double w = c->gs_w[a] * c->gs_w[b] * c->gs_w[e] * c->gs_w[f] * jac;
                        double xr[3], nx[3], yr[3], ny[3], d[3];
                        curved_eval(X, x1, x2, xr, nx);
                        curved_eval(Y, y1, y2, yr, ny);
                        /* X0 = Y0: the shared vertex */
                        for (int k = 0; k < 3; ++k) d[k] = xr[k] - yr[k];
                        double g = w * vnorm(nx) * curved_kernel(op, d, ny, sgn);
                        double lp[3] = {1.0 - x1, x1 - x2, x2}, lq[3] = {1.0 - y1, y1 - y2, y2};
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) M[3 * pa[i] + pb[j]] += g * lp[i] * lq[j];
                    }
}

void orc_curved_moments_many(void *p, int op, int64_t m, const int64_t *I, const int64_t *J, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < m; ++k) orc_curved_moments(p, op, I[k], J[k], out + 9 * k);
}

/* int_t phi_a = int_that l_a gamma by the collapsed rule of order q (area: the sum) */
void orc_curved_mass(void *p, int64_t t, int q, double *m3)
{
    const orc_curved *c = (const orc_curved *)p;
    orc_trirule r;
    rule_collapsed(q, &r);
    int id[3] = {0, 1, 2};
    double X[6][3];
    curved_nodes(c, t, id, X);
    m3[0] = m3[1] = m3[2] = 0.0;
    for (int a = 0; a < r.np; ++a) {
        double xr[3], n[3];
        curved_eval(X, r.s1[a], r.s2[a], xr, n);
        double w = r.w[a] * vnorm(n);
        m3[0] += w * (1.0 - r.s1[a]);
        m3[1] += w * (r.s1[a] - r.s2[a]);
        m3[2] += w * r.s2[a];
    }
}
