/*
 * FP64 CPU oracle of the ligand-pocket docking search (test infrastructure).
 *
 * This file is test infrastructure, not product code: only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant with the GPU path.  It is deliberately plain and
 * slow: every candidate pose is scored from scratch with the definition of the
 * score, in double precision, in the order the method states its steps.
 *
 * The method (paper Sec. 3.1, "The dock and score algorithm"): a ligand has six
 * rigid degrees of freedom plus its torsional bonds, each of which splits the
 * atoms into two sets that turn about the bond axis.  Docking is a greedy
 * optimisation with multiple restarts (one restart per initial orientation),
 * flexible ligand, rigid pocket, driven by a purely geometric (steric) score;
 * the ligand's score is the score of its best pose.  The paper does not define
 * the score, the restarts or the moves further; the synthetic stand-ins used
 * here are:
 *
 *   score  E(X) = sum_i g(X_i, t_i) + penalty * #{ i<j : bonddist(i,j) >= 4,
 *                                                   |X_i - X_j|^2 < cutoff^2 }
 *          g = trilinear interpolation in the per-atom-type grid of the pocket
 *          (node-centred texels, coordinates clamped to the grid).
 *   restarts  K Fibonacci-sphere orientations R_k = Rz(phi_k) Ry(beta_k),
 *          z_k = 1 - (2k+1)/K, beta_k = acos z_k, phi_k = k*pi*(3 - sqrt 5),
 *          placed at the pocket centre: X = c + R_k (X0 - mean X0).
 *   moves  per pass: every rotatable bond in list order (torsional bonds are
 *          serial, Sec. 3.1), S-1 relative turns 2*pi*s/S of the side away from
 *          atom 0, keep the best if strictly better; then, when T = 27, the 26
 *          rigid offsets step*(a,b,c), a,b,c in {-1,0,1}, a slowest, keep the
 *          best if strictly better.  Lower score is better.
 *
 * Ties keep the current pose, then the lower candidate index, then the lower
 * orientation index.  The keep candidates are never re-scored: they reuse the
 * cached score.
 *
 * Oracle-only bookkeeping (used to accept ties inside the tolerance): at every
 * decision the effective gap between the chosen candidate and every other
 * candidate, minus the clash pairs whose distance is within amb_delta of the
 * cutoff (those may count either way in another precision), is compared with
 * tol = near_rel * max(|E|, 1); an orientation with a smaller gap is flagged
 * "near tie".
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

#define ORC_PI 3.14159265358979323846

typedef struct {
    int nx, ny, nz, channels;
    double h;
    double origin[3];
    const float *values; /* [channels][nz][ny][nx], x fastest */
} orc_grid;

typedef struct {
    int n_orient;        /* K */
    int torsion_steps;   /* S */
    int passes;          /* P */
    int n_offsets;       /* T: 1 or 27 */
    double offset_step;  /* A */
    double clash_cutoff; /* A */
    double clash_penalty;
    double near_rel;     /* near-tie relative tolerance */
    double amb_delta;    /* A, clash-distance ambiguity band */
} orc_params;

/* ------------------------------------------------------------------------- */
/* Score: trilinear texel term                                                */
/* ------------------------------------------------------------------------- */

static double texel(const orc_grid *g, int c, int i, int j, int k)
{
    size_t idx = (((size_t)c * g->nz + (size_t)k) * g->ny + (size_t)j) * g->nx + (size_t)i;
    return (double)g->values[idx];
}

static void axis_cell(double x, double o, double h, int nn, int *i, double *f)
{
    double u = (x - o) / h;
    if (u < 0.0) u = 0.0;
    if (u > (double)(nn - 1)) u = (double)(nn - 1);
    double fl = floor(u);
    if (fl > (double)(nn - 2)) fl = (double)(nn - 2);
    *i = (int)fl;
    *f = u - fl;
}

/* g(x, c): product-of-weights trilinear interpolation over the 8 corners. */
double orc_grid_value(const orc_grid *g, int c, const double p[3])
{
    int ix, iy, iz;
    double fx, fy, fz;
    axis_cell(p[0], g->origin[0], g->h, g->nx, &ix, &fx);
    axis_cell(p[1], g->origin[1], g->h, g->ny, &iy, &fy);
    axis_cell(p[2], g->origin[2], g->h, g->nz, &iz, &fz);
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
                s += w * texel(g, c, ix + dx, iy + dy, iz + dz);
            }
    return s;
}

/* ------------------------------------------------------------------------- */
/* Topology                                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, nb, nrot;
    double *x0;           /* [n*3] input conformation, centred on its centroid */
    int *type;            /* [n] */
    int *dist;            /* [n*n] bond-count distance, -1 = unreachable */
    int *rot_u, *rot_v;   /* [nrot] u on atom 0's side */
    unsigned char *moving;/* [nrot*n] 1 = turns with bond b (side of v, without v) */
} orc_lig;

static void lig_free(orc_lig *L)
{
    free(L->x0); free(L->type); free(L->dist);
    free(L->rot_u); free(L->rot_v); free(L->moving);
    memset(L, 0, sizeof(*L));
}

/* BFS over the bond graph from `src`, not crossing the edge (cu, cv) when cu >= 0. */
static void bfs(int n, int nb, const int *bij, int src, int cu, int cv, int *d, int *queue)
{
    for (int i = 0; i < n; ++i) d[i] = -1;
    int head = 0, tail = 0;
    d[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int a = queue[head++];
        for (int e = 0; e < nb; ++e) {
            int p = bij[2 * e], q = bij[2 * e + 1];
            if (cu >= 0 && ((p == cu && q == cv) || (p == cv && q == cu))) continue;
            int o = -1;
            if (p == a) o = q; else if (q == a) o = p;
            if (o >= 0 && d[o] < 0) { d[o] = d[a] + 1; queue[tail++] = o; }
        }
    }
}

/* Bond-count distances (-1 = unreachable) between every pair of atoms. */
int orc_bond_distances(int n, int nb, const int *bij, int *dist)
{
    int *q = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!q) return ORC_ENOMEM;
    for (int e = 0; e < 2 * nb; ++e)
        if (bij[e] < 0 || bij[e] >= n) { free(q); return ORC_EINVAL; }
    for (int i = 0; i < n; ++i) bfs(n, nb, bij, i, -1, -1, dist + (size_t)i * n, q);
    free(q);
    return ORC_OK;
}

/* Orient a rotatable bond (u on atom 0's side) and mark the atoms that turn
 * with it: those reached from v without crossing the bond, v excluded.
 * Fails when the bond is not a bridge (ring bond) or atom 0 is on neither side. */
int orc_moving_set(int n, int nb, const int *bij, int bond, int *u_out, int *v_out,
                   unsigned char *moving)
{
    if (bond < 0 || bond >= nb) return ORC_EINVAL;
    int p = bij[2 * bond], q = bij[2 * bond + 1];
    int *d = (int *)malloc(sizeof(int) * (size_t)n * 2);
    if (!d) return ORC_ENOMEM;
    int *queue = d + n;
    bfs(n, nb, bij, 0, p, q, d, queue);
    int u, v;
    if (d[p] >= 0 && d[q] < 0) { u = p; v = q; }
    else if (d[q] >= 0 && d[p] < 0) { u = q; v = p; }
    else { free(d); return ORC_EINVAL; }
    bfs(n, nb, bij, v, p, q, d, queue);
    for (int i = 0; i < n; ++i) moving[i] = (unsigned char)(d[i] >= 0 && i != v);
    free(d);
    *u_out = u;
    *v_out = v;
    return ORC_OK;
}

static int lig_prepare(orc_lig *L, int n, const float *x, const float *y, const float *z,
                       const unsigned char *type, int nb, const int *bij, int nrot,
                       const int *rot_bond, int channels)
{
    memset(L, 0, sizeof(*L));
    if (n < 1) return ORC_EINVAL;
    L->n = n; L->nb = nb; L->nrot = nrot;
    L->x0 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    L->type = (int *)malloc(sizeof(int) * (size_t)n);
    L->dist = (int *)malloc(sizeof(int) * (size_t)n * n);
    L->rot_u = (int *)malloc(sizeof(int) * (size_t)(nrot > 0 ? nrot : 1));
    L->rot_v = (int *)malloc(sizeof(int) * (size_t)(nrot > 0 ? nrot : 1));
    L->moving = (unsigned char *)malloc((size_t)(nrot > 0 ? nrot : 1) * n);
    if (!L->x0 || !L->type || !L->dist || !L->rot_u || !L->rot_v || !L->moving) {
        lig_free(L);
        return ORC_ENOMEM;
    }
    double c[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        c[0] += (double)x[i]; c[1] += (double)y[i]; c[2] += (double)z[i];
    }
    for (int a = 0; a < 3; ++a) c[a] /= (double)n;
    for (int i = 0; i < n; ++i) {
        L->x0[3 * i + 0] = (double)x[i] - c[0];
        L->x0[3 * i + 1] = (double)y[i] - c[1];
        L->x0[3 * i + 2] = (double)z[i] - c[2];
        if ((int)type[i] >= channels) { lig_free(L); return ORC_EINVAL; }
        L->type[i] = (int)type[i];
    }
    int rc = orc_bond_distances(n, nb, bij, L->dist);
    if (rc) { lig_free(L); return rc; }
    for (int b = 0; b < nrot; ++b) {
        rc = orc_moving_set(n, nb, bij, rot_bond[b], &L->rot_u[b], &L->rot_v[b],
                            L->moving + (size_t)b * n);
        if (rc) { lig_free(L); return rc; }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Score E(X) = grid term + clash term                                        */
/* ------------------------------------------------------------------------- */

typedef struct { double e; int clashes; int ambiguous; } orc_energy;

static orc_energy energy(const orc_grid *g, const orc_lig *L, const orc_params *prm, const double *X)
{
    orc_energy r = {0.0, 0, 0};
    for (int i = 0; i < L->n; ++i) r.e += orc_grid_value(g, L->type[i], X + 3 * i);
    double cut2 = prm->clash_cutoff * prm->clash_cutoff;
    for (int i = 0; i < L->n; ++i)
        for (int j = i + 1; j < L->n; ++j) {
            int d = L->dist[(size_t)i * L->n + j];
            if (d >= 0 && d <= 3) continue;          /* 1-2, 1-3, 1-4 pairs excluded */
            double dx = X[3 * i] - X[3 * j], dy = X[3 * i + 1] - X[3 * j + 1],
                   dz = X[3 * i + 2] - X[3 * j + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < cut2) r.clashes++;
            if (fabs(sqrt(d2) - prm->clash_cutoff) < prm->amb_delta) r.ambiguous++;
        }
    r.e += prm->clash_penalty * (double)r.clashes;
    return r;
}

/* ------------------------------------------------------------------------- */
/* Moves                                                                      */
/* ------------------------------------------------------------------------- */

/* K Fibonacci-sphere rotations: R_k = Rz(phi_k) Ry(beta_k), row-major. */
void orc_orientation(int k, int K, double R[9])
{
    double zk = 1.0 - (2.0 * k + 1.0) / (double)K;
    double beta = acos(zk);
    double phi = (double)k * ORC_PI * (3.0 - sqrt(5.0));
    double cb = cos(beta), sb = sin(beta), cp = cos(phi), sp = sin(phi);
    double Rz[9] = {cp, -sp, 0.0, sp, cp, 0.0, 0.0, 0.0, 1.0};
    double Ry[9] = {cb, 0.0, sb, 0.0, 1.0, 0.0, -sb, 0.0, cb};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int t = 0; t < 3; ++t) s += Rz[3 * r + t] * Ry[3 * t + c];
            R[3 * r + c] = s;
        }
}

/* Rodrigues rotation of the marked atoms about the axis through X_u -> X_v. */
void orc_rotate_about_bond(int n, double *X, int u, int v, const unsigned char *moving, double alpha)
{
    double a[3] = {X[3 * v] - X[3 * u], X[3 * v + 1] - X[3 * u + 1], X[3 * v + 2] - X[3 * u + 2]};
    double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= len; a[1] /= len; a[2] /= len;
    double ca = cos(alpha), sa = sin(alpha);
    for (int i = 0; i < n; ++i) {
        if (!moving[i]) continue;
        double r[3] = {X[3 * i] - X[3 * v], X[3 * i + 1] - X[3 * v + 1], X[3 * i + 2] - X[3 * v + 2]};
        double axr[3] = {a[1] * r[2] - a[2] * r[1], a[2] * r[0] - a[0] * r[2], a[0] * r[1] - a[1] * r[0]};
        double adr = a[0] * r[0] + a[1] * r[1] + a[2] * r[2];
        for (int t = 0; t < 3; ++t)
            X[3 * i + t] = X[3 * v + t] + r[t] * ca + axr[t] * sa + a[t] * adr * (1.0 - ca);
    }
}

static void place(const orc_lig *L, const double R[9], const double centre[3], double *X)
{
    for (int i = 0; i < L->n; ++i) {
        const double *p = L->x0 + 3 * i;
        for (int r = 0; r < 3; ++r)
            X[3 * i + r] = centre[r] + (R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2]);
    }
}

static void grid_centre(const orc_grid *g, double c[3])
{
    c[0] = g->origin[0] + g->h * (double)(g->nx - 1) / 2.0;
    c[1] = g->origin[1] + g->h * (double)(g->ny - 1) / 2.0;
    c[2] = g->origin[2] + g->h * (double)(g->nz - 1) / 2.0;
}

static void offset_of(int o, int abc[3])
{
    abc[0] = o / 9 - 1;
    abc[1] = (o / 3) % 3 - 1;
    abc[2] = o % 3 - 1;
}

/* ------------------------------------------------------------------------- */
/* Search of one orientation                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    double score;
    int clashes, ambiguous;
    int near_tie;
    double min_gap;     /* smallest effective gap over all decisions */
    double min_cand;    /* smallest score over every candidate evaluated */
    double start_score; /* score right after placement */
    int n_decisions;
} orc_orient_result;

/* Near-tie bookkeeping of one decision: candidates cand[0..m-1], chosen index c. */
static void decision_margin(const orc_energy *cand, int m, int c, const orc_params *prm,
                            orc_orient_result *res)
{
    double tol = prm->near_rel * (fabs(cand[c].e) > 1.0 ? fabs(cand[c].e) : 1.0);
    for (int o = 0; o < m; ++o) {
        if (o == c) continue;
        double gap = (cand[o].e - cand[c].e)
                   - prm->clash_penalty * (double)(cand[o].ambiguous + cand[c].ambiguous);
        if (gap < res->min_gap) res->min_gap = gap;
        if (gap < tol) res->near_tie = 1;
    }
    res->n_decisions++;
}

static int search_orientation(const orc_grid *g, const orc_lig *L, const orc_params *prm, int k,
                              double *X, double *Y, orc_energy *cand,
                              int *theta, int tau[3], orc_orient_result *res, double *trace,
                              int trace_cap)
{
    const int K = prm->n_orient, S = prm->torsion_steps, n = L->n;
    double R[9], centre[3];
    orc_orientation(k, K, R);
    grid_centre(g, centre);
    place(L, R, centre, X);
    orc_energy cur = energy(g, L, prm, X);
    memset(res, 0, sizeof(*res));
    res->min_gap = HUGE_VAL;
    res->min_cand = cur.e;
    res->start_score = cur.e;
    for (int b = 0; b < L->nrot; ++b) theta[b] = 0;
    tau[0] = tau[1] = tau[2] = 0;
    int nt = 0;
    if (trace && nt < trace_cap) trace[nt++] = cur.e;

    for (int pass = 0; pass < prm->passes; ++pass) {
        for (int b = 0; b < L->nrot; ++b) {          /* torsional bonds, serially */
            const unsigned char *mv = L->moving + (size_t)b * n;
            cand[0] = cur;
            int best = 0;
            for (int s = 1; s < S; ++s) {
                memcpy(Y, X, sizeof(double) * 3 * (size_t)n);
                orc_rotate_about_bond(n, Y, L->rot_u[b], L->rot_v[b], mv, 2.0 * ORC_PI * s / S);
                cand[s] = energy(g, L, prm, Y);
                if (cand[s].e < res->min_cand) res->min_cand = cand[s].e;
                if (cand[s].e < cand[best].e) best = s;
            }
            decision_margin(cand, S, best, prm, res);
            if (best != 0) {
                orc_rotate_about_bond(n, X, L->rot_u[b], L->rot_v[b], mv, 2.0 * ORC_PI * best / S);
                cur = cand[best];
                theta[b] = (theta[b] + best) % S;
            }
            if (trace && nt < trace_cap) trace[nt++] = cur.e;
        }
        if (prm->n_offsets > 1) {                    /* rigid translations */
            cand[0] = cur;                            /* slot 0 = keep (offset index 13) */
            int best = 0, best_o = 13;
            int slot = 1, slot_o[27];
            slot_o[0] = 13;
            for (int o = 0; o < 27; ++o) {
                if (o == 13) continue;
                int abc[3];
                offset_of(o, abc);
                for (int i = 0; i < n; ++i)
                    for (int t = 0; t < 3; ++t)
                        Y[3 * i + t] = X[3 * i + t] + prm->offset_step * (double)abc[t];
                cand[slot] = energy(g, L, prm, Y);
                if (cand[slot].e < res->min_cand) res->min_cand = cand[slot].e;
                if (cand[slot].e < cand[best].e) { best = slot; best_o = o; }
                slot_o[slot] = o;
                ++slot;
            }
            (void)slot_o;
            decision_margin(cand, 27, best, prm, res);
            if (best != 0) {
                int abc[3];
                offset_of(best_o, abc);
                for (int i = 0; i < n; ++i)
                    for (int t = 0; t < 3; ++t)
                        X[3 * i + t] = X[3 * i + t] + prm->offset_step * (double)abc[t];
                cur = cand[best];
                for (int t = 0; t < 3; ++t) tau[t] += abc[t];
            }
            if (trace && nt < trace_cap) trace[nt++] = cur.e;
        }
    }
    res->score = cur.e;
    res->clashes = cur.clashes;
    res->ambiguous = cur.ambiguous;
    return nt;
}

/* ------------------------------------------------------------------------- */
/* Public entry points                                                        */
/* ------------------------------------------------------------------------- */

/* Score of one conformation as given (no placement). */
int orc_score(const orc_grid *g, const orc_params *prm, int n, const double *X,
              const unsigned char *type, int nb, const int *bij,
              double *score, int *clashes, int *ambiguous)
{
    orc_lig L;
    memset(&L, 0, sizeof(L));
    L.n = n;
    L.type = (int *)malloc(sizeof(int) * (size_t)n);
    L.dist = (int *)malloc(sizeof(int) * (size_t)n * n);
    if (!L.type || !L.dist) { lig_free(&L); return ORC_ENOMEM; }
    for (int i = 0; i < n; ++i) {
        if ((int)type[i] >= g->channels) { lig_free(&L); return ORC_EINVAL; }
        L.type[i] = type[i];
    }
    int rc = orc_bond_distances(n, nb, bij, L.dist);
    if (rc) { lig_free(&L); return rc; }
    orc_energy e = energy(g, &L, prm, X);
    *score = e.e;
    if (clashes) *clashes = e.clashes;
    if (ambiguous) *ambiguous = e.ambiguous;
    lig_free(&L);
    return ORC_OK;
}

/* Pose from its descriptor: X = c + step*tau + R_k FK_theta(X0 - mean X0), where
 * FK_theta turns each rotatable bond's moving set by theta_b*2*pi/S about its
 * current axis, in list order. */
int orc_pose_from_desc(const orc_grid *g, const orc_params *prm, int n, const float *x,
                       const float *y, const float *z, const unsigned char *type, int nb,
                       const int *bij, int nrot, const int *rot_bond, int k, const int *theta,
                       const int tau[3], double *X)
{
    orc_lig L;
    int rc = lig_prepare(&L, n, x, y, z, type, nb, bij, nrot, rot_bond, g->channels);
    if (rc) return rc;
    double *Y = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!Y) { lig_free(&L); return ORC_ENOMEM; }
    memcpy(Y, L.x0, sizeof(double) * 3 * (size_t)n);
    for (int b = 0; b < nrot; ++b)
        if (theta[b] % prm->torsion_steps)
            orc_rotate_about_bond(n, Y, L.rot_u[b], L.rot_v[b], L.moving + (size_t)b * n,
                                  2.0 * ORC_PI * (double)theta[b] / (double)prm->torsion_steps);
    double R[9], c[3];
    orc_orientation(k, prm->n_orient, R);
    grid_centre(g, c);
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < 3; ++r)
            X[3 * i + r] = c[r] + (R[3 * r] * Y[3 * i] + R[3 * r + 1] * Y[3 * i + 1]
                                   + R[3 * r + 2] * Y[3 * i + 2])
                         + prm->offset_step * (double)tau[r];
    free(Y);
    lig_free(&L);
    return ORC_OK;
}

/* The near-tie bookkeeping of one decision, exposed for tests: candidate scores e[m] with
 * their ambiguous clash-pair counts amb[m] (NULL = none), chosen candidate c.  *near_tie = 1
 * when the effective gap to some other candidate is below near_rel * max(|e[c]|, 1);
 * *min_gap = the smallest effective gap (HUGE_VAL when m = 1). */
int orc_decision_margin(int m, const double *e, const int *amb, int c, double near_rel,
                        double clash_penalty, double *min_gap, int *near_tie)
{
    if (m < 1 || c < 0 || c >= m || !e) return ORC_EINVAL;
    orc_energy *cand = (orc_energy *)malloc(sizeof(orc_energy) * (size_t)m);
    if (!cand) return ORC_ENOMEM;
    for (int o = 0; o < m; ++o) {
        cand[o].e = e[o];
        cand[o].clashes = 0;
        cand[o].ambiguous = amb ? amb[o] : 0;
    }
    orc_params prm;
    memset(&prm, 0, sizeof(prm));
    prm.near_rel = near_rel;
    prm.clash_penalty = clash_penalty;
    orc_orient_result res;
    memset(&res, 0, sizeof(res));
    res.min_gap = HUGE_VAL;
    decision_margin(cand, m, c, &prm, &res);
    if (min_gap) *min_gap = res.min_gap;
    if (near_tie) *near_tie = res.near_tie;
    free(cand);
    return ORC_OK;
}

/* Orientation and moving sets of every rotatable bond (exposed for tests). */
int orc_rot_topology(int n, int nb, const int *bij, int nrot, const int *rot_bond,
                     int *u, int *v, unsigned char *moving)
{
    for (int b = 0; b < nrot; ++b) {
        int rc = orc_moving_set(n, nb, bij, rot_bond[b], &u[b], &v[b], moving + (size_t)b * n);
        if (rc) return rc;
    }
    return ORC_OK;
}

/*
 * Dock one ligand: search every orientation.  Outputs (any may be NULL):
 *   score[K], clashes[K], ambiguous[K], near_tie[K], min_gap[K], min_cand[K],
 *   start[K], theta[K*nrot], tau[K*3], coords[K*n*3] (final pose of every
 *   orientation), trace[K*trace_cap] (score after every decision, NaN-padded).
 * best_k / best_score: argmin over orientations, ties to the lower index.
 */
int orc_dock_ligand(const orc_grid *g, const orc_params *prm, int n, const float *x,
                    const float *y, const float *z, const unsigned char *type, int nb,
                    const int *bij, int nrot, const int *rot_bond,
                    double *score, int *clashes, int *ambiguous, int *near_tie, double *min_gap,
                    double *min_cand, double *start, int *theta, int *tau, double *coords,
                    double *trace, int trace_cap, int *best_k, double *best_score)
{
    if (prm->n_orient < 1 || prm->torsion_steps < 1 || prm->passes < 0 ||
        (prm->n_offsets != 1 && prm->n_offsets != 27) || g->nx < 2 || g->ny < 2 || g->nz < 2)
        return ORC_EINVAL;
    orc_lig L;
    int rc = lig_prepare(&L, n, x, y, z, type, nb, bij, nrot, rot_bond, g->channels);
    if (rc) return rc;
    int S = prm->torsion_steps;
    int mc = S > 27 ? S : 27;
    double *X = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *Y = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_energy *cand = (orc_energy *)malloc(sizeof(orc_energy) * (size_t)mc);
    int *th = (int *)malloc(sizeof(int) * (size_t)(nrot > 0 ? nrot : 1));
    if (!X || !Y || !cand || !th) {
        free(X); free(Y); free(cand); free(th); lig_free(&L);
        return ORC_ENOMEM;
    }
    int bk = -1;
    double bs = HUGE_VAL;
    for (int k = 0; k < prm->n_orient; ++k) {
        orc_orient_result res;
        int tu[3];
        double *tr = trace ? trace + (size_t)k * trace_cap : NULL;
        int nt = search_orientation(g, &L, prm, k, X, Y, cand, th, tu, &res, tr, trace_cap);
        if (tr) for (int t = nt; t < trace_cap; ++t) tr[t] = NAN;
        if (score) score[k] = res.score;
        if (clashes) clashes[k] = res.clashes;
        if (ambiguous) ambiguous[k] = res.ambiguous;
        if (near_tie) near_tie[k] = res.near_tie;
        if (min_gap) min_gap[k] = res.min_gap;
        if (min_cand) min_cand[k] = res.min_cand;
        if (start) start[k] = res.start_score;
        if (theta) for (int b = 0; b < nrot; ++b) theta[(size_t)k * nrot + b] = th[b];
        if (tau) for (int t = 0; t < 3; ++t) tau[3 * k + t] = tu[t];
        if (coords) memcpy(coords + (size_t)k * n * 3, X, sizeof(double) * 3 * (size_t)n);
        if (res.score < bs) { bs = res.score; bk = k; }
    }
    if (best_k) *best_k = bk;
    if (best_score) *best_score = bs;
    free(X); free(Y); free(cand); free(th);
    lig_free(&L);
    return ORC_OK;
}

/*
 * Dock a CSR batch of ligands against a set of pockets, OpenMP over ligands.
 * Per ligand l: best_k[l], best_score[l]; per (l, k): score[l*K+k], near_tie[l*K+k],
 * theta[(rot_offset[l]*K) + k*nrot_l + b], tau[(l*K+k)*3 + t]  (any may be NULL).
 * Returns the first error code met (ligands after an error are still docked).
 */
int orc_dock_batch(const orc_grid *grids, int n_grids, const orc_params *prm, int n_lig,
                   const int *atom_offset, const float *x, const float *y, const float *z,
                   const unsigned char *type, const int *bond_offset, const int *bond_ij,
                   const int *rot_offset, const int *rot_bond, const int *pocket_id,
                   int *best_k, double *best_score, double *score, int *near_tie,
                   int *theta, int *tau, int n_threads)
{
    int err = ORC_OK;
    const int K = prm->n_orient;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
    for (int l = 0; l < n_lig; ++l) {
        int a0 = atom_offset[l], n = atom_offset[l + 1] - a0;
        int b0 = bond_offset[l], nb = bond_offset[l + 1] - b0;
        int r0 = rot_offset[l], nr = rot_offset[l + 1] - r0;
        int pid = pocket_id ? pocket_id[l] : 0;
        if (pid < 0 || pid >= n_grids) {
#pragma omp critical
            err = ORC_EINVAL;
            continue;
        }
        int bk = -1;
        double bs = 0.0;
        int rc = orc_dock_ligand(&grids[pid], prm, n, x + a0, y + a0, z + a0, type + a0, nb,
                                 bond_ij + 2 * (size_t)b0, nr, rot_bond + r0,
                                 score ? score + (size_t)l * K : NULL, NULL, NULL,
                                 near_tie ? near_tie + (size_t)l * K : NULL, NULL, NULL, NULL,
                                 theta ? theta + (size_t)r0 * K : NULL,
                                 tau ? tau + (size_t)l * K * 3 : NULL, NULL, NULL, 0, &bk, &bs);
        if (rc) {
#pragma omp critical
            err = rc;
        }
        if (best_k) best_k[l] = bk;
        if (best_score) best_score[l] = bs;
    }
    return err;
}

/* ------------------------------------------------------------------------- */
/* Ranking of the final poses (third step of the method)                    */
/* ------------------------------------------------------------------------- */

/*
 * Sec. 3.1, third step: the generated poses of a ligand are clustered with an
 * RMSD threshold (two poses are similar when their RMSD is below it), then
 * listed with the best-scoring pose of every cluster first and all the other
 * poses after them, each group by the (geometric) score.  The paper names
 * neither the RMSD nor the clustering procedure; the readings are:
 *   RMSD(a, b) = sqrt(mean_i |a_i - b_i|^2) over all atoms, same frame (no
 *            superposition: the poses share the pocket's frame);
 *   clusters  greedy leaders: poses taken by score (lower first, ties to the
 *            lower orientation index); a pose starts a new cluster (is a
 *            leader) unless its RMSD to some earlier leader is below thr.
 * A leader is then the best-scoring pose of its cluster.
 */
double orc_rmsd(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < 3 * n; ++i) {
        double d = a[i] - b[i];
        s += d * d;
    }
    return sqrt(s / (double)n);
}

/* poses [K][n][3], scores [K].  Out: order [K] (pose indices, leaders by score
 * then the others by score), leader [K] (1 for a leader).  Returns the number of
 * leaders (or < 0 on bad arguments).  Oracle bookkeeping: *amb_rmsd counts the
 * leader tests whose RMSD lies within delta of thr; *amb_score counts pairs of
 * poses adjacent in score order whose scores differ by less than
 * tol * max(|s|, 1) (either may be taken first in another precision). */
int orc_rank_poses(int K, int n, const double *poses, const double *scores, double thr,
                   double delta, double tol, int *order, int *leader, int *amb_rmsd,
                   int *amb_score)
{
    if (K < 1 || n < 1 || !poses || !scores || !order || !leader) return ORC_EINVAL;
    int *by_score = (int *)malloc(sizeof(int) * (size_t)K);
    int *leaders = (int *)malloc(sizeof(int) * (size_t)K);
    if (!by_score || !leaders) { free(by_score); free(leaders); return ORC_ENOMEM; }
    /* 1. poses by score: insertion sort on (score, index), NaN last */
    for (int k = 0; k < K; ++k) {
        int j = k;
        double s = scores[k];
        while (j > 0) {
            int p = by_score[j - 1];
            double sp = scores[p];
            int before = isnan(s) ? 0 : (isnan(sp) ? 1 : (s < sp));   /* k before p? */
            if (!before) break;
            by_score[j] = p;
            --j;
        }
        by_score[j] = k;
    }
    int ns = 0;
    for (int j = 0; j + 1 < K; ++j) {
        double a = scores[by_score[j]], b = scores[by_score[j + 1]];
        double m = fabs(a) > 1.0 ? fabs(a) : 1.0;
        if (fabs(a - b) < tol * m) ++ns;
    }
    /* 2. greedy leaders */
    int nl = 0, nr = 0;
    for (int j = 0; j < K; ++j) {
        int p = by_score[j];
        int similar = 0;
        for (int q = 0; q < nl; ++q) {
            double r = orc_rmsd(n, poses + (size_t)p * n * 3, poses + (size_t)leaders[q] * n * 3);
            if (fabs(r - thr) < delta) ++nr;
            if (r < thr) similar = 1;
        }
        leader[p] = !similar;
        if (!similar) leaders[nl++] = p;
    }
    /* 3. leaders by score, then the others by score */
    int o = 0;
    for (int j = 0; j < K; ++j) if (leader[by_score[j]]) order[o++] = by_score[j];
    for (int j = 0; j < K; ++j) if (!leader[by_score[j]]) order[o++] = by_score[j];
    if (amb_rmsd) *amb_rmsd = nr;
    if (amb_score) *amb_score = ns;
    free(by_score);
    free(leaders);
    return nl;
}

/* ------------------------------------------------------------------------- */
/* Unfolding of the input conformation (first step of the method)           */
/* ------------------------------------------------------------------------- */

/*
 * Sec. 3.1, first step: before docking, and independently of the protein, the
 * ligand is flattened by turning its torsional bonds so that the sum of the
 * distances between all its atoms is as large as possible.  The paper gives no
 * procedure; the reading here mirrors the docking sweep: per pass, every
 * rotatable bond in list order tries the S-1 relative turns 2*pi*s/S of the side
 * without atom 0 and keeps the largest sum if strictly larger (ties keep the
 * current shape, then the lower s).
 */
double orc_distance_sum(int n, const double *X)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dx = X[3 * i] - X[3 * j], dy = X[3 * i + 1] - X[3 * j + 1],
                   dz = X[3 * i + 2] - X[3 * j + 2];
            s += sqrt(dx * dx + dy * dy + dz * dz);
        }
    return s;
}

/* Input conformation x, y, z (A), bonds, rotatable bonds.  Out: X_out [n*3] in the input
 * frame (atom 0's side does not move), turns [passes*nrot] (the s kept per pass and bond),
 * *near_ties = decisions where another turn's sum is within tol * m * (n - m) of the kept one,
 * m the atoms that turn with the bond: a turn changes only the m * (n - m) distances between
 * turning and fixed atoms, so tol is a per-distance allowance (A) for another precision. */
int orc_unfold_ligand(int n, const float *x, const float *y, const float *z, int nb,
                      const int *bij, int nrot, const int *rot_bond, int S, int passes,
                      double tol, double *X_out, int *turns, int *near_ties)
{
    if (n < 1 || S < 1 || passes < 0 || !X_out) return ORC_EINVAL;
    int *u = (int *)malloc(sizeof(int) * (size_t)(nrot > 0 ? nrot : 1));
    int *v = (int *)malloc(sizeof(int) * (size_t)(nrot > 0 ? nrot : 1));
    unsigned char *mv = (unsigned char *)malloc((size_t)(nrot > 0 ? nrot : 1) * n);
    double *Y = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *cand = (double *)malloc(sizeof(double) * (size_t)S);
    int rc = ORC_OK, nt = 0;
    if (!u || !v || !mv || !Y || !cand) { rc = ORC_ENOMEM; goto done; }
    for (int b = 0; b < nrot; ++b) {
        rc = orc_moving_set(n, nb, bij, rot_bond[b], &u[b], &v[b], mv + (size_t)b * n);
        if (rc) goto done;
    }
    for (int i = 0; i < n; ++i) {
        X_out[3 * i] = (double)x[i]; X_out[3 * i + 1] = (double)y[i]; X_out[3 * i + 2] = (double)z[i];
    }
    for (int p = 0; p < passes; ++p)
        for (int b = 0; b < nrot; ++b) {
            cand[0] = orc_distance_sum(n, X_out);
            for (int s = 1; s < S; ++s) {
                memcpy(Y, X_out, sizeof(double) * 3 * (size_t)n);
                orc_rotate_about_bond(n, Y, u[b], v[b], mv + (size_t)b * n, 2.0 * ORC_PI * s / S);
                cand[s] = orc_distance_sum(n, Y);
            }
            int best = 0;
            for (int s = 1; s < S; ++s)
                if (cand[s] > cand[best]) best = s;
            int nm = 0;
            for (int i = 0; i < n; ++i) nm += mv[(size_t)b * n + i];
            double band = tol * (double)nm * (double)(n - nm);
            for (int s = 0; s < S; ++s)
                if (s != best && cand[best] - cand[s] < band) { ++nt; break; }
            if (best != 0)
                orc_rotate_about_bond(n, X_out, u[b], v[b], mv + (size_t)b * n, 2.0 * ORC_PI * best / S);
            if (turns) turns[p * nrot + b] = best;
        }
done:
    if (near_ties) *near_ties = nt;
    free(u); free(v); free(mv); free(Y); free(cand);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Second-stage rescoring of the ranked poses (Sec. 3.1, fourth step)         */
/* ------------------------------------------------------------------------- */

/*
 * The paper rescores the first 30 poses of each ligand's ranked list with a
 * richer chemical score (LiGen's), which it does not define.  The stand-in
 * score of a pose X (FP64, plain definition):
 *
 *   E2(X) = sum_i g(X_i, t_i)                                  pocket grid term
 *         + sum_{i<j, bonddist(i,j) >= 4 or unbonded}
 *               eps * ((s/d')^12 - 2 (s/d')^6),  d' = max(d_ij, s/2)
 *                                                              smooth contact term,
 *                                                              minimum -eps at d = s
 *         + sum_b w * (1 + cos 3 phi_b)                        threefold torsional strain
 *
 * with s the clash cutoff.  phi_b is the dihedral a-i-j-c of rotatable bond b
 * = (i, j) as listed in the bond list, a the lowest-index neighbour of i other
 * than j, c the lowest-index neighbour of j other than i; a bond without such a
 * or c, or whose dihedral is undefined (|(X_i - X_a) x (X_j - X_i)| or
 * |(X_j - X_i) x (X_c - X_j)| below 1e-9 A^2), contributes nothing.  The dihedral
 * does not depend on which end is listed first.  parts (may be NULL) receives
 * the three terms.
 */
int orc_rescore2(const orc_grid *g, int n, const double *X, const unsigned char *type, int nb,
                 const int *bij, int nrot, const int *rot_bond, double sigma, double eps,
                 double w, double *e2, double parts[3])
{
    if (n < 1 || !X || !type || !e2) return ORC_EINVAL;
    int *dist = (int *)malloc(sizeof(int) * (size_t)n * n);
    if (!dist) return ORC_ENOMEM;
    int rc = orc_bond_distances(n, nb, bij, dist);
    if (rc) { free(dist); return rc; }
    double grid = 0.0, contact = 0.0, tors = 0.0;
    for (int i = 0; i < n; ++i) {
        if ((int)type[i] >= g->channels) { free(dist); return ORC_EINVAL; }
        grid += orc_grid_value(g, type[i], X + 3 * i);
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int d = dist[(size_t)i * n + j];
            if (d >= 0 && d <= 3) continue;
            double dx = X[3 * i] - X[3 * j], dy = X[3 * i + 1] - X[3 * j + 1],
                   dz = X[3 * i + 2] - X[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r < 0.5 * sigma) r = 0.5 * sigma;
            double q = sigma / r;
            double q6 = q * q * q * q * q * q;
            contact += eps * (q6 * q6 - 2.0 * q6);
        }
    for (int b = 0; b < nrot; ++b) {
        if (rot_bond[b] < 0 || rot_bond[b] >= nb) { free(dist); return ORC_EINVAL; }
        int i = bij[2 * rot_bond[b]], j = bij[2 * rot_bond[b] + 1];
        int a = -1, c = -1;
        for (int k = 0; k < n; ++k) {
            if (a < 0 && k != j && dist[(size_t)i * n + k] == 1) a = k;
            if (c < 0 && k != i && dist[(size_t)j * n + k] == 1) c = k;
        }
        if (a < 0 || c < 0) continue;
        double b1[3], b2[3], b3[3];
        for (int t = 0; t < 3; ++t) {
            b1[t] = X[3 * i + t] - X[3 * a + t];
            b2[t] = X[3 * j + t] - X[3 * i + t];
            b3[t] = X[3 * c + t] - X[3 * j + t];
        }
        double n1[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
                        b1[0] * b2[1] - b1[1] * b2[0]};
        double n2[3] = {b2[1] * b3[2] - b2[2] * b3[1], b2[2] * b3[0] - b2[0] * b3[2],
                        b2[0] * b3[1] - b2[1] * b3[0]};
        double l1 = sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
        double l2 = sqrt(n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
        if (l1 < 1e-9 || l2 < 1e-9) continue;
        double cph = (n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]) / (l1 * l2);
        if (cph > 1.0) cph = 1.0;
        if (cph < -1.0) cph = -1.0;
        double phi = acos(cph);
        tors += w * (1.0 + cos(3.0 * phi));
    }
    free(dist);
    *e2 = grid + contact + tors;
    if (parts) { parts[0] = grid; parts[1] = contact; parts[2] = tors; }
    return ORC_OK;
}
