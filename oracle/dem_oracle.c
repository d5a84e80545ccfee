/*
 * dem_oracle.c -- plain FP64 CPU oracle for the rounded-polytope DEM method
 * of Spellings, Marson, Anderson & Glotzer (arXiv:1607.02427).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the library never does, and the
 * two share no code, headers, tables or helpers.
 *
 * What it computes, in the paper's terms:
 *   - Pair energy (Sec. II, Eq. 1 in 3D, Eq. 2 in 2D): the sum of a point
 *     potential over every edge-edge and vertex-face feature pair (3D) or
 *     every vertex-edge pair (2D), each evaluated at the nearest points of the
 *     two features.  Every feature pair is brute-forced; nothing is culled
 *     except particle pairs whose centres are farther apart than
 *     R_i + R_j + r_cut (then no feature pair can reach the cutoff).
 *   - Point potential (Sec. II, Eq. 3 and Eq. 4): WCA, the Lennard-Jones
 *     potential shifted by its value at r_cut = 2^(1/6) sigma and cut there,
 *     with sigma_ij = r_i + r_j (the surface sits sigma/2 from the features).
 *   - Force along the nearest-point line, torque about each particle's centre
 *     from that particle's own nearest point (Sec. II, after Eq. 2).
 *   - Nearly parallel edges: the interaction points are the midpoints of the
 *     edges' mutual overlap (Sec. II, the paragraph after Eq. 4).
 *   - Molecular virial W = sum_{i<j} r_ij (x) F_ij (Sec. IV.C names a virial
 *     tensor for the barostat; the definition used is the standard one).
 *   - Cell list and full neighbour list (the paper relies on its host MD
 *     framework for these; the reading used here is the plain definition).
 *   - Second-order rigid-body integrator (Sec. IV.A) and a Nose-Hoover
 *     thermostat on translation and rotation (Sec. IV.C): velocity Verlet for
 *     the centre of mass, a symmetric split of free rotations about the
 *     principal axes for the orientation, a Trotter-wrapped Nose-Hoover half
 *     step before and after.
 *
 * Readings where the paper is silent are listed in the design notes of the
 * repository; each is marked at its use below.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 * -ffp-contract=off matters: the list decisions must be the plain IEEE
 * evaluation of the stated expressions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXV 64
#define OR_TWO_POW_SIXTH 1.122462048309373 /* 2^(1/6) to double precision */

typedef struct {
    int dim;
    int n_shapes;
    const int *nv, *ne, *nf;        /* per shape counts */
    const int *v_off, *e_off, *f_off; /* per shape first index (n_shapes+1) */
    const double *verts;            /* [total_v][3] body frame */
    const int *edges;               /* [total_e][2] local vertex ids */
    const int *fl_off;              /* [total_f+1] offsets into floops */
    const int *floops;              /* local vertex ids, CCW from outside */
    const double *rad;              /* rounding radius per shape */
    const double *mass;             /* per shape */
    const double *inertia;          /* [n_shapes][3] principal moments */
    double box[3];
    double epsilon;
    double par_s2;                  /* parallel threshold on sin^2 */
} or_sys;

typedef struct {
    double U;          /* pair energy U_ij */
    double Fi[3];      /* force on i */
    double Ti[3];      /* torque on i about x_i */
    double Tj[3];      /* torque on j about its image x_j' */
    double W[9];       /* (x_i - x_j') (x) F_i, row-major */
    double Fabs, Tabs_i, Wabs; /* sums of |f|, |(P - x_i) x f|, |r_ij (x) f| over feature pairs */
    int n_in;          /* feature pairs inside the cutoff */
    int n_par;         /* of those, evaluated with the parallel rule */
    int n_near_par;    /* of those, within +-1% of the parallel threshold */
} or_pair_out;

/* ---------------------------------------------------------------- vectors */
static inline void v_sub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static inline double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void v_cross(const double *a, const double *b, double *o)
{
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static inline void v_axpy(double s, const double *x, const double *y, double *o) { o[0] = y[0] + s * x[0]; o[1] = y[1] + s * x[1]; o[2] = y[2] + s * x[2]; }

/* Rotation matrix (row-major) of a unit quaternion (w, x, y, z), body -> space. */
static void quat_to_mat(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
static inline void mat_vec(const double *R, const double *v, double *o)
{
    double t0 = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    double t1 = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    double t2 = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static inline void matT_vec(const double *R, const double *v, double *o)
{
    double t0 = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
    double t1 = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
    double t2 = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
    o[0] = t0; o[1] = t1; o[2] = t2;
}

/* ----------------------------------------------------------- WCA (Eq. 3-4) */
/* For r^2 < r_cut^2 returns 1 and sets U (Eq. 4: U_LJ(r) - U_LJ(r_cut);
 * U_LJ(r_cut) = -eps exactly, so the shift is +eps) and fr = -dU/dr / r, so
 * that the force on the first point is fr * (P - Q).  Otherwise returns 0. */
int or_wca(double r2, double sigma, double eps, double *U, double *fr)
{
    double rc = OR_TWO_POW_SIXTH * sigma;
    if (!(r2 < rc * rc)) { *U = 0.0; *fr = 0.0; return 0; }
    double s2 = sigma * sigma / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    *U = 4.0 * eps * (s12 - s6) + eps;
    *fr = 24.0 * eps * (2.0 * s12 - s6) / r2;
    return 1;
}

/* ------------------------------------------------- nearest-point primitives */
/* Point-segment (Sec. II: "standard point-line formula"): the closed segment
 * [a, b]; t = clamp((p-a).(b-a)/|b-a|^2, 0, 1). */
void or_point_segment(const double *p, const double *a, const double *b, double *q)
{
    double u[3], w[3];
    v_sub(b, a, u);
    v_sub(p, a, w);
    double t = v_dot(w, u) / v_dot(u, u);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    v_axpy(t, u, a, q);
}

/* Segment-segment closest points (Sec. II: "line-line formula").
 * Non-parallel: f(s,t) = |a0 + s u - b0 - t v|^2 is strictly convex on the
 * unit square, so its minimum is the interior stationary point if that lies
 * in [0,1]^2, else the best of the four boundary problems, each a
 * point-segment projection.  Ties keep the first candidate.
 * Nearly parallel, |u x v|^2 < par_s2 |u|^2 |v|^2 (threshold reading): each
 * point is the midpoint of its segment's overlap with the other segment's
 * projection onto its line; with no overlap, the endpoint facing the other
 * segment (Sec. II, the paragraph on parallel edges).
 * Returns 1 when the parallel rule was used. */
int or_segment_segment(const double *a0, const double *a1, const double *b0, const double *b1,
                       double par_s2, double *P, double *Q)
{
    double u[3], v[3], w[3], c[3];
    v_sub(a1, a0, u);
    v_sub(b1, b0, v);
    v_sub(a0, b0, w);
    double A = v_dot(u, u), C = v_dot(v, v);
    v_cross(u, v, c);
    double den = v_dot(c, c);
    if (den < par_s2 * A * C) {
        double t0, t1, lo, hi, d0[3], d1[3];
        /* overlap on segment a */
        v_sub(b0, a0, d0);
        v_sub(b1, a0, d1);
        t0 = v_dot(d0, u) / A;
        t1 = v_dot(d1, u) / A;
        lo = fmax(0.0, fmin(t0, t1));
        hi = fmin(1.0, fmax(t0, t1));
        double sa = (lo <= hi) ? 0.5 * (lo + hi) : (fmax(t0, t1) < 0.0 ? 0.0 : 1.0);
        /* overlap on segment b */
        v_sub(a0, b0, d0);
        v_sub(a1, b0, d1);
        t0 = v_dot(d0, v) / C;
        t1 = v_dot(d1, v) / C;
        lo = fmax(0.0, fmin(t0, t1));
        hi = fmin(1.0, fmax(t0, t1));
        double sb = (lo <= hi) ? 0.5 * (lo + hi) : (fmax(t0, t1) < 0.0 ? 0.0 : 1.0);
        v_axpy(sa, u, a0, P);
        v_axpy(sb, v, b0, Q);
        return 1;
    }
    double B = v_dot(u, v), D = v_dot(u, w), E = v_dot(v, w);
    double s = (B * E - C * D) / den;
    double t = (A * E - B * D) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
        v_axpy(s, u, a0, P);
        v_axpy(t, v, b0, Q);
        return 0;
    }
    /* boundary: four point-segment problems */
    double best = INFINITY, cp[3], cq[3], d[3], r2;
    or_point_segment(a0, b0, b1, cq);
    v_sub(a0, cq, d); r2 = v_dot(d, d);
    if (r2 < best) { best = r2; memcpy(P, a0, sizeof cp); memcpy(Q, cq, sizeof cq); }
    or_point_segment(a1, b0, b1, cq);
    v_sub(a1, cq, d); r2 = v_dot(d, d);
    if (r2 < best) { best = r2; memcpy(P, a1, sizeof cp); memcpy(Q, cq, sizeof cq); }
    or_point_segment(b0, a0, a1, cp);
    v_sub(cp, b0, d); r2 = v_dot(d, d);
    if (r2 < best) { best = r2; memcpy(P, cp, sizeof cp); memcpy(Q, b0, sizeof cq); }
    or_point_segment(b1, a0, a1, cp);
    v_sub(cp, b1, d); r2 = v_dot(d, d);
    if (r2 < best) { best = r2; memcpy(P, cp, sizeof cp); memcpy(Q, b1, sizeof cq); }
    return 0;
}

/* Returns 1 if the segment pair is within +-1% of the parallel threshold. */
static int near_parallel(const double *a0, const double *a1, const double *b0, const double *b1, double par_s2)
{
    double u[3], v[3], c[3];
    v_sub(a1, a0, u);
    v_sub(b1, b0, v);
    v_cross(u, v, c);
    double lhs = v_dot(c, c), rhs = par_s2 * v_dot(u, u) * v_dot(v, v);
    return lhs > 0.99 * rhs && lhs < 1.01 * rhs;
}

/* Point to closed planar polygon (Sec. II: "point-plane formula").  The loop
 * (k points, xyz) may be concave.  Project onto the plane; if the projection
 * is inside (crossing-number test in face coordinates) it is the nearest
 * point, otherwise the nearest point lies on the polygon's own edges. */
static int point_polygon(const double *p, const double *loop, int k, double *q);

void or_point_polygon(const double *p, const double *loop, int k, double *q) { (void)point_polygon(p, loop, k, q); }

/* The nearest point as above; returns 1 when the projection lies inside
 * the polygon (the nearest point is the projection), 0 when it lies on the
 * polygon's edges. */
static int point_polygon(const double *p, const double *loop, int k, double *q)
{
    double n[3] = {0, 0, 0};
    for (int a = 0; a < k; ++a) { /* Newell normal */
        const double *s = loop + 3 * a, *t = loop + 3 * ((a + 1) % k);
        double c[3];
        v_cross(s, t, c);
        n[0] += c[0]; n[1] += c[1]; n[2] += c[2];
    }
    double nn = sqrt(v_dot(n, n));
    n[0] /= nn; n[1] /= nn; n[2] /= nn;
    double w[3];
    v_sub(p, loop, w);
    double sd = v_dot(w, n);
    double pr[3];
    v_axpy(-sd, n, p, pr);
    /* face coordinates */
    double e1[3], e2[3];
    v_sub(loop + 3, loop, e1);
    double l1 = sqrt(v_dot(e1, e1));
    e1[0] /= l1; e1[1] /= l1; e1[2] /= l1;
    v_cross(n, e1, e2);
    double px, py;
    {
        double d[3];
        v_sub(pr, loop, d);
        px = v_dot(d, e1);
        py = v_dot(d, e2);
    }
    int inside = 0;
    for (int a = 0; a < k; ++a) {
        double d0[3], d1[3];
        v_sub(loop + 3 * a, loop, d0);
        v_sub(loop + 3 * ((a + 1) % k), loop, d1);
        double x0 = v_dot(d0, e1), y0 = v_dot(d0, e2);
        double x1 = v_dot(d1, e1), y1 = v_dot(d1, e2);
        if ((y0 > py) != (y1 > py)) {
            double xc = x0 + (py - y0) * (x1 - x0) / (y1 - y0);
            if (px < xc) inside = !inside;
        }
    }
    if (inside) { memcpy(q, pr, 3 * sizeof(double)); return 1; }
    double best = INFINITY;
    for (int a = 0; a < k; ++a) {
        double c[3], d[3];
        or_point_segment(p, loop + 3 * a, loop + 3 * ((a + 1) % k), c);
        v_sub(p, c, d);
        double r2 = v_dot(d, d);
        if (r2 < best) { best = r2; memcpy(q, c, sizeof c); }
    }
    return 0;
}

/* ------------------------------------------------------------ pair energy */
/* One feature pair inside the cutoff, for diagnostics (or_pair_terms):
 * family 0 = E_i-E_j (a, b edges of i and j), 1 = V_i-F_j (a vertex of i, b
 * face of j), 2 = V_j-F_i (a vertex of j, b face of i), 3 = 2D V_i-E_j,
 * 4 = 2D V_j-E_i, 5 = point-point (spheres, disks); inside = 1 when a vertex-face nearest point is the
 * projection onto the face, 0 when it lies on the face's edges, -1 for the
 * other families; par = the parallel-edge rule applied; r = |P - Q|. */
typedef struct {
    int family, a, b, inside, par;
    double r;
} or_term;

typedef struct {
    or_term *buf;
    int cap, n;
} or_terms;

static void note(or_terms *t, int family, int a, int b, int inside, int par, double r)
{
    if (!t) return;
    if (t->n < t->cap) {
        or_term *e = t->buf + t->n;
        e->family = family; e->a = a; e->b = b; e->inside = inside; e->par = par; e->r = r;
    }
    t->n += 1;
}

/* Adds the term of nearest points P (on i) and Q (on j) when |P - Q| is
 * inside the cutoff; returns |P - Q| then, else -1. */
static double accumulate(or_pair_out *o, const double *P, const double *Q, const double *xi, const double *xj,
                         double sigma, double eps, int par, int near_par)
{
    double rho[3];
    v_sub(P, Q, rho);
    double U, fr;
    if (!or_wca(v_dot(rho, rho), sigma, eps, &U, &fr)) return -1.0;
    double f[3] = {fr * rho[0], fr * rho[1], fr * rho[2]};
    double ai[3], aj[3], ti[3], tj[3], rij[3];
    v_sub(P, xi, ai);
    v_sub(Q, xj, aj);
    v_cross(ai, f, ti);
    v_cross(aj, f, tj); /* torque on j is aj x (-f) */
    v_sub(xi, xj, rij);
    o->U += U;
    o->Fabs += sqrt(v_dot(f, f));
    o->Tabs_i += sqrt(v_dot(ti, ti));
    o->Wabs += sqrt(v_dot(rij, rij)) * sqrt(v_dot(f, f));
    for (int k = 0; k < 3; ++k) {
        o->Fi[k] += f[k];
        o->Ti[k] += ti[k];
        o->Tj[k] -= tj[k];
        for (int l = 0; l < 3; ++l) o->W[3 * k + l] += rij[k] * f[l];
    }
    o->n_in += 1;
    o->n_par += par;
    o->n_near_par += near_par;
    return sqrt(v_dot(rho, rho));
}

/* Full evaluation of U_ij and its derivatives for particles of shapes si, sj
 * at positions xi, xj (xj already the image nearest to xi) and quaternions.
 * 3D: Eq. 1 (every E_i-E_j pair, every V_i-F_j pair, every V_j-F_i pair);
 * 2D: Eq. 2 (every V_i-E_j pair and every V_j-E_i pair).  A shape that is a
 * single point (no edges, no faces) is a sphere (2D: a disk) of radius r:
 * against a polytope it enters Eq. 1/2 as one vertex; two of them interact
 * by the central WCA potential of Eq. 3/4 at the distance of their points,
 * the spheres of Sec. IV.B (family 5). */
static void pair_eval(const or_sys *S, int si, int sj, const double *xi, const double *qi, const double *xj,
                      const double *qj, or_pair_out *o, or_terms *tl)
{
    memset(o, 0, sizeof *o);
    double Ri[9], Rj[9];
    quat_to_mat(qi, Ri);
    quat_to_mat(qj, Rj);
    double Vi[OR_MAXV][3], Vj[OR_MAXV][3];
    int nvi = S->nv[si], nvj = S->nv[sj];
    for (int k = 0; k < nvi; ++k) {
        double t[3];
        mat_vec(Ri, S->verts + 3 * (S->v_off[si] + k), t);
        Vi[k][0] = xi[0] + t[0]; Vi[k][1] = xi[1] + t[1]; Vi[k][2] = xi[2] + t[2];
    }
    for (int k = 0; k < nvj; ++k) {
        double t[3];
        mat_vec(Rj, S->verts + 3 * (S->v_off[sj] + k), t);
        Vj[k][0] = xj[0] + t[0]; Vj[k][1] = xj[1] + t[1]; Vj[k][2] = xj[2] + t[2];
    }
    double sigma = S->rad[si] + S->rad[sj];
    double eps = S->epsilon;
    const int *Ei = S->edges + 2 * S->e_off[si], *Ej = S->edges + 2 * S->e_off[sj];
    int nei = S->ne[si], nej = S->ne[sj];
    if (nei == 0 && nej == 0 && S->nf[si] == 0 && S->nf[sj] == 0) {
        for (int a = 0; a < nvi; ++a)
            for (int b = 0; b < nvj; ++b) {
                double r = accumulate(o, Vi[a], Vj[b], xi, xj, sigma, eps, 0, 0);
                if (r >= 0.0) note(tl, 5, a, b, -1, 0, r);
            }
        return;
    }
    if (S->dim == 2) {
        for (int a = 0; a < nvi; ++a)
            for (int e = 0; e < nej; ++e) {
                double q[3];
                or_point_segment(Vi[a], Vj[Ej[2 * e]], Vj[Ej[2 * e + 1]], q);
                double r = accumulate(o, Vi[a], q, xi, xj, sigma, eps, 0, 0);
                if (r >= 0.0) note(tl, 3, a, e, -1, 0, r);
            }
        for (int b = 0; b < nvj; ++b)
            for (int e = 0; e < nei; ++e) {
                double p[3];
                or_point_segment(Vj[b], Vi[Ei[2 * e]], Vi[Ei[2 * e + 1]], p);
                double r = accumulate(o, p, Vj[b], xi, xj, sigma, eps, 0, 0);
                if (r >= 0.0) note(tl, 4, b, e, -1, 0, r);
            }
        return;
    }
    for (int e = 0; e < nei; ++e)
        for (int g = 0; g < nej; ++g) {
            double P[3], Q[3];
            const double *a0 = Vi[Ei[2 * e]], *a1 = Vi[Ei[2 * e + 1]];
            const double *b0 = Vj[Ej[2 * g]], *b1 = Vj[Ej[2 * g + 1]];
            int par = or_segment_segment(a0, a1, b0, b1, S->par_s2, P, Q);
            double r = accumulate(o, P, Q, xi, xj, sigma, eps, par, near_parallel(a0, a1, b0, b1, S->par_s2));
            if (r >= 0.0) note(tl, 0, e, g, -1, par, r);
        }
    double loop[OR_MAXV * 3];
    for (int a = 0; a < nvi; ++a)
        for (int f = 0; f < S->nf[sj]; ++f) {
            int gf = S->f_off[sj] + f, k = S->fl_off[gf + 1] - S->fl_off[gf];
            for (int c = 0; c < k; ++c) memcpy(loop + 3 * c, Vj[S->floops[S->fl_off[gf] + c]], 3 * sizeof(double));
            double q[3];
            int in = point_polygon(Vi[a], loop, k, q);
            double r = accumulate(o, Vi[a], q, xi, xj, sigma, eps, 0, 0);
            if (r >= 0.0) note(tl, 1, a, f, in, 0, r);
        }
    for (int b = 0; b < nvj; ++b)
        for (int f = 0; f < S->nf[si]; ++f) {
            int gf = S->f_off[si] + f, k = S->fl_off[gf + 1] - S->fl_off[gf];
            for (int c = 0; c < k; ++c) memcpy(loop + 3 * c, Vi[S->floops[S->fl_off[gf] + c]], 3 * sizeof(double));
            double p[3];
            int in = point_polygon(Vj[b], loop, k, p);
            double r = accumulate(o, p, Vj[b], xi, xj, sigma, eps, 0, 0);
            if (r >= 0.0) note(tl, 2, b, f, in, 0, r);
        }
}

void or_pair(const or_sys *S, int si, int sj, const double *xi, const double *qi, const double *xj,
             const double *qj, or_pair_out *o)
{
    pair_eval(S, si, sj, xi, qi, xj, qj, o, NULL);
}

/* The same evaluation, listing the feature pairs inside the cutoff (at most
 * cap of them into terms); returns how many there are.  A diagnostic for
 * the tests: which families and which branch of the point-polygon rule a
 * case reaches. */
int or_pair_terms(const or_sys *S, int si, int sj, const double *xi, const double *qi, const double *xj,
                  const double *qj, or_term *terms, int cap)
{
    or_pair_out o;
    or_terms t = {terms, cap, 0};
    pair_eval(S, si, sj, xi, qi, xj, qj, &o, &t);
    return t.n;
}

/* ------------------------------------------------------------ geometry */
static double shape_R(const or_sys *S, int s)
{
    double R = 0.0;
    for (int k = 0; k < S->nv[s]; ++k) {
        const double *v = S->verts + 3 * (S->v_off[s] + k);
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (r > R) R = r;
    }
    return R;
}

/* Neighbour-list radius: 2 R_max + r_cut(sigma_max) + skin. */
double or_r_list(const or_sys *S, double skin)
{
    double Rm = 0.0, rm = 0.0;
    for (int s = 0; s < S->n_shapes; ++s) {
        double R = shape_R(S, s);
        if (R > Rm) Rm = R;
        if (S->rad[s] > rm) rm = S->rad[s];
    }
    return 2.0 * Rm + OR_TWO_POW_SIXTH * (2.0 * rm) + skin;
}

static inline double min_image(double d, double L) { return d - L * rint(d / L); }

/* ---------------------------------------------------- cell and nbr lists */
/* Cells per axis: floor(L / r_list); 2D uses one layer in z. */
void or_cell_dims(const or_sys *S, double r_list, int *nc)
{
    for (int a = 0; a < 3; ++a) nc[a] = (a < S->dim) ? (int)floor(S->box[a] / r_list) : 1;
}

static int cell_coord(double x, double L, int n)
{
    double w = L / (double)n;
    int c = (int)floor(x / w);
    if (c < 0) c = 0;
    if (c > n - 1) c = n - 1;
    return c;
}

/* CSR cell list: cell_start[ncells+1], cell_particles[n] ascending within a
 * cell.  Linear cell index c = cx + nx (cy + ny cz).  Returns ncells. */
int or_cell_list(const or_sys *S, int n, const double *x, double r_list, int *cell_start, int *cell_particles)
{
    int nc[3];
    or_cell_dims(S, r_list, nc);
    int ncell = nc[0] * nc[1] * nc[2];
    if (ncell < 1) return 0;
    int *cid = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    memset(cell_start, 0, sizeof(int) * (size_t)(ncell + 1));
    for (int i = 0; i < n; ++i) {
        int c[3] = {0, 0, 0};
        for (int a = 0; a < S->dim; ++a) c[a] = cell_coord(x[3 * i + a], S->box[a], nc[a]);
        cid[i] = c[0] + nc[0] * (c[1] + nc[1] * c[2]);
        cell_start[cid[i] + 1] += 1;
    }
    for (int c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    for (int i = 0; i < n; ++i) { /* ascending i, so each cell stays sorted */
        int c = cid[i];
        cell_particles[cell_start[c] + fill[c]] = i;
        fill[c] += 1;
    }
    free(fill);
    free(cid);
    return ncell;
}

static int cmp_int(const void *a, const void *b) { int x = *(const int *)a, y = *(const int *)b; return (x > y) - (x < y); }

/* Is j a neighbour of i: |minimum image (x_j - x_i)|^2 < r_list^2, evaluated
 * as ((dx*dx + dy*dy) + dz*dz) with no contraction. */
static int within(const or_sys *S, const double *x, int i, int j, double rl2)
{
    double r2 = 0.0;
    for (int a = 0; a < S->dim; ++a) {
        double d = min_image(x[3 * j + a] - x[3 * i + a], S->box[a]);
        r2 = r2 + d * d;
    }
    return r2 < rl2;
}

/* Full neighbour list, rows ascending in j, ELL column-major nbr[k*n + i].
 * mode 0: all pairs; mode 1: the 3^d cells around i's cell (requires at
 * least 3 cells per periodic axis; falls back to all pairs otherwise).
 * Returns the largest row length (rows longer than cap are truncated). */
int or_nbr_list(const or_sys *S, int n, const double *x, double r_list, int cap, int mode, int *nbr, int *n_nbr)
{
    double rl2 = r_list * r_list;
    int nc[3];
    or_cell_dims(S, r_list, nc);
    int use_cells = (mode == 1);
    for (int a = 0; a < S->dim; ++a)
        if (nc[a] < 3) use_cells = 0;
    int ncell = nc[0] * nc[1] * nc[2];
    int *cs = NULL, *cp = NULL;
    if (use_cells) {
        cs = (int *)malloc(sizeof(int) * (size_t)(ncell + 1));
        cp = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
        or_cell_list(S, n, x, r_list, cs, cp);
    }
    int maxrow = 0;
    int *row = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        int m = 0;
        if (use_cells) {
            int c[3] = {0, 0, 0};
            for (int a = 0; a < S->dim; ++a) c[a] = cell_coord(x[3 * i + a], S->box[a], nc[a]);
            int zlo = (S->dim == 3) ? -1 : 0, zhi = (S->dim == 3) ? 1 : 0;
            for (int dz = zlo; dz <= zhi; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cx = (c[0] + dx + nc[0]) % nc[0];
                        int cy = (c[1] + dy + nc[1]) % nc[1];
                        int cz = (c[2] + dz + nc[2]) % nc[2];
                        int cc = cx + nc[0] * (cy + nc[1] * cz);
                        for (int t = cs[cc]; t < cs[cc + 1]; ++t) {
                            int j = cp[t];
                            if (j != i && within(S, x, i, j, rl2)) row[m++] = j;
                        }
                    }
        } else {
            for (int j = 0; j < n; ++j)
                if (j != i && within(S, x, i, j, rl2)) row[m++] = j;
        }
        qsort(row, (size_t)m, sizeof(int), cmp_int);
        if (m > maxrow) maxrow = m;
        int mm = m < cap ? m : cap;
        for (int k = 0; k < mm; ++k) nbr[(size_t)k * n + i] = row[k];
        n_nbr[i] = mm;
    }
    free(row);
    free(cs);
    free(cp);
    return maxrow;
}

/* ------------------------------------------------------------- forces */
typedef struct {
    long n_pairs_bound;   /* ordered pairs within R_i + R_j + r_cut */
    long n_feature_in;    /* feature pairs inside the cutoff (ordered) */
    long n_par;
    long n_near_par;
} or_stats;

/* Per-particle force F_i, torque tau_i, energy U_i = 1/2 sum_j U_ij and
 * virial W_i = 1/2 sum_j (x_i - x_j) (x) F_ij.  Each particle sums its own
 * interactions over every other particle (mode 0) or over its cell-list
 * neighbours (mode 1); particle pairs farther apart than R_i + R_j + r_cut
 * are skipped because no feature pair can then reach the cutoff. */
static void forces_of(const or_sys *S, int n, const double *x, const double *q, const int *sid, int mode,
                      const int *pick, int m_pick, double *F, double *T, double *U, double *W, or_stats *st,
                      double *scale);

void or_forces(const or_sys *S, int n, const double *x, const double *q, const int *sid, int mode,
               double *F, double *T, double *U, double *W, or_stats *st, double *scale)
{
    forces_of(S, n, x, q, sid, mode, NULL, n, F, T, U, W, st, scale);
}

/* The same sums for the m particles pick[0..m) only (each against every
 * other particle of the system); output row k belongs to particle pick[k]. */
void or_forces_subset(const or_sys *S, int n, const double *x, const double *q, const int *sid, int mode,
                      const int *pick, int m, double *F, double *T, double *U, double *W, or_stats *st,
                      double *scale)
{
    forces_of(S, n, x, q, sid, mode, pick, m, F, T, U, W, st, scale);
}

static void forces_of(const or_sys *S, int n, const double *x, const double *q, const int *sid, int mode,
                      const int *pick, int m_pick, double *F, double *T, double *U, double *W, or_stats *st,
                      double *scale)
{
    double R[64];
    for (int s = 0; s < S->n_shapes && s < 64; ++s) R[s] = shape_R(S, s);
    double rmax = 0.0, Rmax = 0.0;
    for (int s = 0; s < S->n_shapes; ++s) { if (S->rad[s] > rmax) rmax = S->rad[s]; if (R[s] > Rmax) Rmax = R[s]; }
    double bound_max = 2.0 * Rmax + OR_TWO_POW_SIXTH * 2.0 * rmax;
    int *nbr = NULL, *n_nbr = NULL;
    if (mode == 1) {
        int cap = 128;
        for (;;) {
            nbr = (int *)malloc(sizeof(int) * (size_t)cap * (size_t)(n > 0 ? n : 1));
            n_nbr = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
            int maxrow = or_nbr_list(S, n, x, bound_max, cap, 1, nbr, n_nbr);
            if (maxrow <= cap) break;
            free(nbr);
            free(n_nbr);
            cap = maxrow;
        }
    }
    long c_pairs = 0, c_in = 0, c_par = 0, c_near = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : c_pairs, c_in, c_par, c_near)
    for (int row = 0; row < m_pick; ++row) {
        const int i = pick ? pick[row] : row;
        double Fi[3] = {0, 0, 0}, Ti[3] = {0, 0, 0}, Ui = 0.0, Wi[9] = {0}, sF = 0.0, sT = 0.0, sW = 0.0;
        int m = (mode == 1) ? n_nbr[i] : n;
        for (int k = 0; k < m; ++k) {
            int j = (mode == 1) ? nbr[(size_t)k * n + i] : k;
            if (j == i) continue;
            double d[3] = {0, 0, 0};
            for (int a = 0; a < S->dim; ++a) d[a] = min_image(x[3 * j + a] - x[3 * i + a], S->box[a]);
            int si = sid[i], sj = sid[j];
            double bound = R[si] + R[sj] + OR_TWO_POW_SIXTH * (S->rad[si] + S->rad[sj]);
            if (v_dot(d, d) >= bound * bound) continue;
            double xj[3] = {x[3 * i] + d[0], x[3 * i + 1] + d[1], x[3 * i + 2] + d[2]};
            or_pair_out o;
            or_pair(S, si, sj, x + 3 * i, q + 4 * i, xj, q + 4 * j, &o);
            c_pairs += 1;
            c_in += o.n_in;
            c_par += o.n_par;
            c_near += o.n_near_par;
            for (int a = 0; a < 3; ++a) { Fi[a] += o.Fi[a]; Ti[a] += o.Ti[a]; }
            Ui += 0.5 * o.U;
            for (int a = 0; a < 9; ++a) Wi[a] += 0.5 * o.W[a];
            sF += o.Fabs;
            sT += o.Tabs_i;
            sW += 0.5 * o.Wabs;
        }
        if (scale) {
            scale[3 * row] = sF;
            scale[3 * row + 1] = sT;
            scale[3 * row + 2] = sW;
        }
        for (int a = 0; a < 3; ++a) { F[3 * row + a] = Fi[a]; T[3 * row + a] = Ti[a]; }
        U[row] = Ui;
        for (int a = 0; a < 9; ++a) W[9 * row + a] = Wi[a];
    }
    if (st) { st->n_pairs_bound = c_pairs; st->n_feature_in = c_in; st->n_par = c_par; st->n_near_par = c_near; }
    free(nbr);
    free(n_nbr);
}

/* ----------------------------------------------------------- integrator */
static void quat_mul(const double *a, const double *b, double *o)
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

/* Free rotation about body axis k for time h: the body turns by
 * phi = h L_k / I_k, so q <- q (x) (cos phi/2, sin phi/2 e_k) and the
 * body-frame angular momentum turns by -phi about e_k. */
static void free_rot(double *q, double *L, const double *I, int k, double h)
{
    if (I[k] <= 0.0) return;
    double phi = h * L[k] / I[k];
    double r[4] = {cos(0.5 * phi), 0, 0, 0};
    r[1 + k] = sin(0.5 * phi);
    double t[4];
    quat_mul(q, r, t);
    memcpy(q, t, sizeof t);
    double c = cos(phi), s = sin(phi);
    int a = (k + 1) % 3, b = (k + 2) % 3; /* cyclic: rotation by -phi maps (La, Lb) */
    double La = L[a], Lb = L[b];
    L[a] = c * La + s * Lb;
    L[b] = -s * La + c * Lb;
}

static void kinetic(const or_sys *S, int n, const double *v, const double *L, const int *sid, double *Kt, double *Kr)
{
    double kt = 0.0, kr = 0.0;
    for (int i = 0; i < n; ++i) {
        double m = S->mass[sid[i]];
        const double *I = S->inertia + 3 * sid[i];
        kt += 0.5 * m * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
        for (int k = 0; k < 3; ++k)
            if (I[k] > 0.0) kr += 0.5 * L[3 * i + k] * L[3 * i + k] / I[k];
    }
    *Kt = kt;
    *Kr = kr;
}

/* Nose-Hoover half step of length h on one variable xi coupled to both
 * translation and rotation (g degrees of freedom, mass Qm). */
static void nh_half(const or_sys *S, int n, double *v, double *L, const int *sid, double h, double g, double kT,
                    double Qm, double *xi, double *eta)
{
    double Kt, Kr;
    kinetic(S, n, v, L, sid, &Kt, &Kr);
    double K = Kt + Kr;
    *xi += 0.5 * h * (2.0 * K - g * kT) / Qm;
    double s = exp(-(*xi) * h);
    for (int i = 0; i < 3 * n; ++i) { v[i] *= s; L[i] *= s; }
    K *= s * s;
    *eta += (*xi) * h;
    *xi += 0.5 * h * (2.0 * K - g * kT) / Qm;
}

/* Runs n_steps of velocity Verlet with the symmetric principal-axis split
 * z(h/2) y(h/2) x(h) y(h/2) z(h/2) for free rotation (3D) or a rotation
 * about z (2D); ensemble 0 = NVE, 1 = NVT.  State arrays are (n,3)/(n,4)
 * row-major and updated in place; thermo = {xi, eta}.  If log is non-NULL it
 * receives per step {U, K_trans, K_rot, xi, eta, H} where H is the total
 * energy (NVE) or the Nose-Hoover conserved quantity (NVT).  Forces use mode
 * (0 all pairs, 1 cell list) and are left in F, T, U, W. */
void or_run(const or_sys *S, int n, double *x, double *q, double *v, double *L, int *image, const int *sid,
            int n_steps, double dt, int ensemble, double kT, double tau_T, double *thermo, int mode, double *F,
            double *T, double *Ui, double *W, double *log)
{
    int d = S->dim, drot = (d == 2) ? 1 : 3;
    double g = (double)(d * n + drot * n - d);
    double Qm = g * kT * tau_T * tau_T;
    double xi = thermo[0], eta = thermo[1];
    or_forces(S, n, x, q, sid, mode, F, T, Ui, W, NULL, NULL);
    for (int step = 0; step < n_steps; ++step) {
        if (ensemble == 1) nh_half(S, n, v, L, sid, 0.5 * dt, g, kT, Qm, &xi, &eta);
        for (int i = 0; i < n; ++i) {
            double m = S->mass[sid[i]];
            double Rm[9], tb[3];
            for (int a = 0; a < d; ++a) v[3 * i + a] += 0.5 * dt * F[3 * i + a] / m;
            quat_to_mat(q + 4 * i, Rm);
            matT_vec(Rm, T + 3 * i, tb);
            if (d == 2) L[3 * i + 2] += 0.5 * dt * T[3 * i + 2];
            else for (int a = 0; a < 3; ++a) L[3 * i + a] += 0.5 * dt * tb[a];
            for (int a = 0; a < d; ++a) {
                double xa = x[3 * i + a] + dt * v[3 * i + a];
                double Lb = S->box[a];
                if (xa >= Lb) { xa -= Lb; image[3 * i + a] += 1; }
                else if (xa < 0.0) { xa += Lb; image[3 * i + a] -= 1; }
                x[3 * i + a] = xa;
            }
            const double *I = S->inertia + 3 * sid[i];
            double *qi = q + 4 * i, *Li = L + 3 * i;
            if (d == 2) {
                free_rot(qi, Li, I, 2, dt);
            } else {
                free_rot(qi, Li, I, 2, 0.5 * dt);
                free_rot(qi, Li, I, 1, 0.5 * dt);
                free_rot(qi, Li, I, 0, dt);
                free_rot(qi, Li, I, 1, 0.5 * dt);
                free_rot(qi, Li, I, 2, 0.5 * dt);
            }
            double qn = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
            for (int a = 0; a < 4; ++a) qi[a] /= qn;
        }
        or_forces(S, n, x, q, sid, mode, F, T, Ui, W, NULL, NULL);
        for (int i = 0; i < n; ++i) {
            double m = S->mass[sid[i]];
            double Rm[9], tb[3];
            for (int a = 0; a < d; ++a) v[3 * i + a] += 0.5 * dt * F[3 * i + a] / m;
            quat_to_mat(q + 4 * i, Rm);
            matT_vec(Rm, T + 3 * i, tb);
            if (d == 2) L[3 * i + 2] += 0.5 * dt * T[3 * i + 2];
            else for (int a = 0; a < 3; ++a) L[3 * i + a] += 0.5 * dt * tb[a];
        }
        if (ensemble == 1) nh_half(S, n, v, L, sid, 0.5 * dt, g, kT, Qm, &xi, &eta);
        if (log) {
            double Kt, Kr, U = 0.0;
            kinetic(S, n, v, L, sid, &Kt, &Kr);
            for (int i = 0; i < n; ++i) U += Ui[i];
            double H = Kt + Kr + U;
            if (ensemble == 1) H += 0.5 * Qm * xi * xi + g * kT * eta;
            double *row = log + 6 * step;
            row[0] = U; row[1] = Kt; row[2] = Kr; row[3] = xi; row[4] = eta; row[5] = H;
        }
    }
    thermo[0] = xi;
    thermo[1] = eta;
}

/* ------------------------------------------------- isothermal-isobaric */
/* Sec. IV.C runs the assembly at fixed pressure with a barostat that takes
 * the pressure from the virial tensor and cites the measure-preserving
 * isothermal-isobaric integrator of Tuckerman et al. (2006).  The reading
 * used here (isotropic box, one Nose-Hoover variable on translation,
 * rotation and the barostat):
 *   d = dimension, N_f = d (N - 1), alpha = 1 + d / N_f,
 *   W = (N_f + d) kT tau_P^2 (barostat mass), g' = g + 1, Q = g' kT tau_T^2,
 *   dx/dt = v + v_eps x,       dv/dt = F/m - (alpha v_eps + xi) v,
 *   dL/dt = tau - xi L (plus the free rotation), dV/dt = d V v_eps,
 *   dv_eps/dt = G_eps / W - xi v_eps,
 *   G_eps = alpha 2 K_trans + tr W_vir - d V P_ext,
 *   dxi/dt = (2 K_trans + 2 K_rot + W v_eps^2 - g' kT) / Q, deta/dt = xi.
 * Conserved: K_trans + K_rot + U + W v_eps^2 / 2 + P_ext V + Q xi^2 / 2
 * + g' kT eta.  One step of length h is the symmetric Trotter sequence
 *   thermostat h/2, barostat h/2, kick h/2, drift h (with the box), free
 *   rotation, forces, kick h/2, barostat h/2, thermostat h/2,
 * where the kick and the drift are the exact flows of their linear parts:
 *   v <- v e^{-alpha v_eps h/2} + (h/2)(F/m) e^{-alpha v_eps h/4} sinhc(alpha v_eps h/4),
 *   x <- x e^{v_eps h} + h v e^{v_eps h/2} sinhc(v_eps h/2),  L_box <- L_box e^{v_eps h},
 * with sinhc(u) = sinh(u) / u.  Positions are then wrapped into the new box. */
static double sinhc(double u)
{
    if (fabs(u) < 1e-3) {
        double u2 = u * u;
        return 1.0 + u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0));
    }
    return sinh(u) / u;
}

static double trace_virial(const or_sys *S, int n, const double *W)
{
    double tr = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < S->dim; ++a) tr += W[9 * i + 4 * a];
    return tr;
}

static double volume(const or_sys *S)
{
    return S->dim == 3 ? S->box[0] * S->box[1] * S->box[2] : S->box[0] * S->box[1];
}

/* Thermostat half step of length h (as nh_half, with the barostat's kinetic
 * term W v_eps^2 in the drive and v_eps scaled with the velocities). */
static void nh_half_npt(const or_sys *S, int n, double *v, double *L, const int *sid, double h, double g, double kT,
                        double Qm, double Wm, double *veps, double *xi, double *eta)
{
    double Kt, Kr;
    kinetic(S, n, v, L, sid, &Kt, &Kr);
    double K2 = 2.0 * (Kt + Kr) + Wm * (*veps) * (*veps);
    *xi += 0.5 * h * (K2 - g * kT) / Qm;
    double s = exp(-(*xi) * h);
    for (int i = 0; i < 3 * n; ++i) { v[i] *= s; L[i] *= s; }
    *veps *= s;
    K2 *= s * s;
    *eta += (*xi) * h;
    *xi += 0.5 * h * (K2 - g * kT) / Qm;
}

static void baro_half(const or_sys *S, int n, const double *v, const double *L, const int *sid, const double *W,
                      double h, double alpha, double Pext, double Wm, double *veps)
{
    double Kt, Kr;
    kinetic(S, n, v, L, sid, &Kt, &Kr);
    double G = alpha * 2.0 * Kt + trace_virial(S, n, W) - S->dim * volume(S) * Pext;
    *veps += h * G / Wm;
}

static void kick_npt(const or_sys *S, int n, double *v, double *L, const double *q, const int *sid, const double *F,
                     const double *T, double h, double alpha, double veps)
{
    int d = S->dim;
    double a = alpha * veps;
    double damp = exp(-a * 0.5 * h), fk = 0.5 * h * exp(-a * 0.25 * h) * sinhc(a * 0.25 * h);
    for (int i = 0; i < n; ++i) {
        double m = S->mass[sid[i]];
        double Rm[9], tb[3];
        for (int c = 0; c < d; ++c) v[3 * i + c] = v[3 * i + c] * damp + fk * F[3 * i + c] / m;
        quat_to_mat(q + 4 * i, Rm);
        matT_vec(Rm, T + 3 * i, tb);
        if (d == 2) L[3 * i + 2] += 0.5 * h * T[3 * i + 2];
        else for (int c = 0; c < 3; ++c) L[3 * i + c] += 0.5 * h * tb[c];
    }
}

/* Runs n_steps of the isothermal-isobaric integrator above.  box[3] is the
 * box (updated), baro[1] = v_eps, thermo = {xi, eta}; log rows, if log is
 * non-NULL: {U, K_trans, K_rot, xi, eta, H, V, P_int, v_eps} with
 * P_int = (2 K_trans + tr W_vir) / (d V). */
void or_run_npt(const or_sys *S0, int n, double *x, double *q, double *v, double *L, int *image, const int *sid,
                int n_steps, double dt, double kT, double tau_T, double Pext, double tau_P, double *box,
                double *thermo, double *baro, int mode, double *F, double *T, double *Ui, double *W, double *log)
{
    or_sys Sl = *S0;
    or_sys *S = &Sl;
    for (int a = 0; a < 3; ++a) S->box[a] = box[a];
    int d = S->dim, drot = (d == 2) ? 1 : 3;
    double g = (double)(d * n + drot * n - d) + 1.0;
    double Nf = (double)(d * (n - 1));
    double alpha = 1.0 + d / Nf;
    double Qm = g * kT * tau_T * tau_T;
    double Wm = (Nf + d) * kT * tau_P * tau_P;
    double xi = thermo[0], eta = thermo[1], veps = baro[0];
    or_forces(S, n, x, q, sid, mode, F, T, Ui, W, NULL, NULL);
    for (int step = 0; step < n_steps; ++step) {
        nh_half_npt(S, n, v, L, sid, 0.5 * dt, g, kT, Qm, Wm, &veps, &xi, &eta);
        baro_half(S, n, v, L, sid, W, 0.5 * dt, alpha, Pext, Wm, &veps);
        kick_npt(S, n, v, L, q, sid, F, T, dt, alpha, veps);
        double grow = exp(veps * dt), vfac = dt * exp(veps * 0.5 * dt) * sinhc(veps * 0.5 * dt);
        for (int a = 0; a < d; ++a) S->box[a] *= grow;
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < d; ++a) {
                double xa = x[3 * i + a] * grow + vfac * v[3 * i + a];
                double Lb = S->box[a];
                if (xa >= Lb) { xa -= Lb; image[3 * i + a] += 1; }
                else if (xa < 0.0) { xa += Lb; image[3 * i + a] -= 1; }
                x[3 * i + a] = xa;
            }
            const double *I = S->inertia + 3 * sid[i];
            double *qi = q + 4 * i, *Li = L + 3 * i;
            if (d == 2) {
                free_rot(qi, Li, I, 2, dt);
            } else {
                free_rot(qi, Li, I, 2, 0.5 * dt);
                free_rot(qi, Li, I, 1, 0.5 * dt);
                free_rot(qi, Li, I, 0, dt);
                free_rot(qi, Li, I, 1, 0.5 * dt);
                free_rot(qi, Li, I, 2, 0.5 * dt);
            }
            double qn = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
            for (int a = 0; a < 4; ++a) qi[a] /= qn;
        }
        or_forces(S, n, x, q, sid, mode, F, T, Ui, W, NULL, NULL);
        kick_npt(S, n, v, L, q, sid, F, T, dt, alpha, veps);
        baro_half(S, n, v, L, sid, W, 0.5 * dt, alpha, Pext, Wm, &veps);
        nh_half_npt(S, n, v, L, sid, 0.5 * dt, g, kT, Qm, Wm, &veps, &xi, &eta);
        if (log) {
            double Kt, Kr, U = 0.0;
            kinetic(S, n, v, L, sid, &Kt, &Kr);
            for (int i = 0; i < n; ++i) U += Ui[i];
            double V = volume(S);
            double H = Kt + Kr + U + 0.5 * Wm * veps * veps + Pext * V + 0.5 * Qm * xi * xi + g * kT * eta;
            double *row = log + 9 * step;
            row[0] = U; row[1] = Kt; row[2] = Kr; row[3] = xi; row[4] = eta; row[5] = H;
            row[6] = V; row[7] = (2.0 * Kt + trace_virial(S, n, W)) / (d * V); row[8] = veps;
        }
    }
    for (int a = 0; a < 3; ++a) box[a] = S->box[a];
    thermo[0] = xi;
    thermo[1] = eta;
    baro[0] = veps;
}

void or_set_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
