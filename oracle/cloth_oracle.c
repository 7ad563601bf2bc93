/*
 * FP64 CPU oracle for the mass-spring cloth step -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load this
 * library.  The product (the HIP library) never calls, links or includes it, and it shares
 * no code with the product: no headers, helpers or tables.  It is deliberately plain and
 * slow: loops written in the order of the method's definition, FP64 throughout, single
 * threaded, no blocking or fusion beyond what the definition states.
 *
 * What one substep computes (h = frame dt / substeps):
 *   1. Spring forces, spring-centric, as in Alg. 1 of the paper's appendix: for a spring
 *      (a, b) with rest length L0, stiffness k and damping c,
 *          dir = normalize(x_b - x_a)
 *          f   = (k (|x_b - x_a| - L0) + c (v_b . dir - v_a . dir)) dir
 *      added to node a and subtracted from node b (action and reaction).
 *   2. Explicit integration (Sec. 3 names an Euler method; read here as semi-implicit
 *      Euler): v* = v + h (w (F + f_ext) + g), x* = x + h v*, with w = 1/m and f_ext an
 *      optional per-node external force (zero unless set).  Pinned nodes (w = 0)
 *      keep x and get v* = 0.
 *   3. Collision against a static triangle surface.  The paper averages a per-collision
 *      direction over all hits of a node (Sec. 3, collision paragraph) and applies it in
 *      Alg. 2: if the node has at least one hit, v <- -0.5 v and pos <- pos + direction.
 *      Here a hit is a triangle t with point-triangle distance dist(x*, t) < th, the
 *      direction of a hit is (th - (x* - A_t) . n_t) n_t with n_t the unit outward normal
 *      (it puts x* at distance th in front of the triangle's plane), the directions are
 *      averaged over the hits, and the restitution factor (0.5 in Alg. 2) is a parameter.
 *   The candidate set is defined by brute force over all triangles; a bucket grid is used
 *   only to skip triangles whose bounding box, inflated by th plus a slack of ORC_BOX_SLACK,
 *   cannot contain x*.  dist < th implies x* lies in that box, so the filter never changes
 *   the result; the slack lets the near-threshold margin see triangles just beyond th.
 *
 * The surface may be moved between substeps (orc_model_set_surface): each substep sees the
 * surface as it was last set.
 *
 * Also here: the FP32 brute-force broad-phase predicate (the exact candidate set a
 * uniform grid must reproduce), the reverse-mode adjoint of one substep with the contact
 * set held fixed, and a checkpointed rollout gradient.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -o libcloth_oracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ small vector helpers */

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ model */

#define ORC_BOX_SLACK 1e-5 /* m: extra inflation of the acceleration boxes */

typedef struct {
    int N, S, V, T;
    double *w;          /* [N] inverse mass, 0 = pinned */
    int *ends;          /* [S][2] */
    double *rest, *k, *c;
    double g[3];
    double *verts;      /* [V][3] */
    int *tris;          /* [T][3] */
    double *fext;       /* [N][3] external forces (NULL = none) */
    double th;          /* collision thickness (0 disables collision) */
    double restitution; /* v <- -restitution v on contact */
    /* per triangle: first vertex, unit outward normal, inflated bounding box */
    double *tA, *tn, *tlo, *thi;
    /* bucket grid over the inflated boxes (acceleration only) */
    double org[3], cell, cell_req;
    int dim[3];
    int *cell_start, *cell_tris;
} orc_model;


static int cell_coord(const orc_model *m, double p, int axis)
{
    double f = floor((p - m->org[axis]) / m->cell);
    if (!(f >= 0.0)) return 0; /* also catches NaN */
    if (f > (double)(m->dim[axis] - 1)) return m->dim[axis] - 1;
    return (int)f;
}

static void build_surface(orc_model *m, double cell)
{
    int T = m->T;
    m->tA = calloc((size_t)T * 3 + 1, sizeof(double));
    m->tn = calloc((size_t)T * 3 + 1, sizeof(double));
    m->tlo = calloc((size_t)T * 3 + 1, sizeof(double));
    m->thi = calloc((size_t)T * 3 + 1, sizeof(double));
    double bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = 0; t < T; ++t) {
        const double *A = m->verts + 3 * m->tris[3 * t + 0];
        const double *B = m->verts + 3 * m->tris[3 * t + 1];
        const double *C = m->verts + 3 * m->tris[3 * t + 2];
        double e1[3], e2[3], n[3];
        sub3(B, A, e1);
        sub3(C, A, e2);
        cross3(e1, e2, n);
        double ln = sqrt(dot3(n, n));
        for (int a = 0; a < 3; ++a) {
            m->tA[3 * t + a] = A[a];
            m->tn[3 * t + a] = n[a] / ln;
            double lo = fmin(A[a], fmin(B[a], C[a])) - m->th - ORC_BOX_SLACK;
            double hi = fmax(A[a], fmax(B[a], C[a])) + m->th + ORC_BOX_SLACK;
            m->tlo[3 * t + a] = lo;
            m->thi[3 * t + a] = hi;
            if (lo < bmin[a]) bmin[a] = lo;
            if (hi > bmax[a]) bmax[a] = hi;
        }
    }
    if (T == 0) {
        m->cell = 1.0;
        for (int a = 0; a < 3; ++a) { m->org[a] = 0; m->dim[a] = 1; }
    } else {
        if (!(cell > 0)) cell = 0.05;
        /* keep the bucket count modest: grow the cell until it holds */
        for (;;) {
            long long tot = 1;
            for (int a = 0; a < 3; ++a) {
                long long d = (long long)floor((bmax[a] - bmin[a]) / cell) + 1;
                tot *= d;
            }
            if (tot <= (1LL << 23)) break;
            cell *= 2.0;
        }
        m->cell = cell;
        for (int a = 0; a < 3; ++a) {
            m->org[a] = bmin[a];
            m->dim[a] = (int)floor((bmax[a] - bmin[a]) / cell) + 1;
        }
    }
    long long ncell = (long long)m->dim[0] * m->dim[1] * m->dim[2];
    m->cell_start = calloc((size_t)ncell + 1, sizeof(int));
    /* count, prefix, fill -- plain counting sort by cell, triangles in ascending id */
    for (int pass = 0; pass < 2; ++pass) {
        int *fill = NULL;
        if (pass == 1) {
            for (long long i = 0; i < ncell; ++i) m->cell_start[i + 1] += m->cell_start[i];
            m->cell_tris = malloc(sizeof(int) * ((size_t)m->cell_start[ncell] + 1));
            fill = calloc((size_t)ncell + 1, sizeof(int));
        }
        for (int t = 0; t < T; ++t) {
            int lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = cell_coord(m, m->tlo[3 * t + a], a);
                hi[a] = cell_coord(m, m->thi[3 * t + a], a);
            }
            for (int i = lo[0]; i <= hi[0]; ++i)
                for (int j = lo[1]; j <= hi[1]; ++j)
                    for (int q = lo[2]; q <= hi[2]; ++q) {
                        long long id = ((long long)q * m->dim[1] + j) * m->dim[0] + i;
                        if (pass == 0) m->cell_start[id + 1] += 1;
                        else m->cell_tris[m->cell_start[id] + fill[id]++] = t;
                    }
        }
        free(fill);
    }
}

orc_model *orc_model_new(int N, const double *w, int S, const int *ends, const double *rest,
                         const double *k, const double *c, const double *g, int V,
                         const double *verts, int T, const int *tris, double th,
                         double restitution, double cell)
{
    orc_model *m = calloc(1, sizeof(orc_model));
    m->N = N; m->S = S; m->V = V; m->T = T;
    m->w = malloc(sizeof(double) * (size_t)(N + 1));
    memcpy(m->w, w, sizeof(double) * (size_t)N);
    m->ends = malloc(sizeof(int) * (size_t)(2 * S + 1));
    memcpy(m->ends, ends, sizeof(int) * (size_t)(2 * S));
    m->rest = malloc(sizeof(double) * (size_t)(S + 1));
    m->k = malloc(sizeof(double) * (size_t)(S + 1));
    m->c = malloc(sizeof(double) * (size_t)(S + 1));
    memcpy(m->rest, rest, sizeof(double) * (size_t)S);
    memcpy(m->k, k, sizeof(double) * (size_t)S);
    memcpy(m->c, c, sizeof(double) * (size_t)S);
    for (int a = 0; a < 3; ++a) m->g[a] = g[a];
    m->verts = malloc(sizeof(double) * (size_t)(3 * V + 1));
    if (V) memcpy(m->verts, verts, sizeof(double) * (size_t)(3 * V));
    m->tris = malloc(sizeof(int) * (size_t)(3 * T + 1));
    if (T) memcpy(m->tris, tris, sizeof(int) * (size_t)(3 * T));
    m->th = th;
    m->restitution = restitution;
    if (th <= 0) m->T = T = 0; /* collision disabled */
    m->cell_req = cell;
    build_surface(m, cell);
    return m;
}

/* Replace the surface's vertex positions (same triangles) and rebuild everything derived
 * from them: a moving or deforming collision surface is a static one between two calls. */
void orc_model_set_surface(orc_model *m, const double *verts)
{
    if (m->V) memcpy(m->verts, verts, sizeof(double) * (size_t)(3 * m->V));
    free(m->tA); free(m->tn); free(m->tlo); free(m->thi);
    free(m->cell_start); free(m->cell_tris);
    m->cell_tris = NULL;
    build_surface(m, m->cell_req);
}

/* External per-node forces f[N][3] (a pull on part of the cloth, Sec. 4's pulled-cloth
 * scenes), added to the spring forces of every node before integration; NULL removes them.
 * Pinned nodes ignore them like any force. */
void orc_model_set_external(orc_model *m, const double *f)
{
    free(m->fext);
    m->fext = NULL;
    if (f) {
        m->fext = malloc(sizeof(double) * 3 * (size_t)(m->N + 1));
        memcpy(m->fext, f, sizeof(double) * 3 * (size_t)m->N);
    }
}

static double fext_of(const orc_model *m, int i, int q) { return m->fext ? m->fext[3 * i + q] : 0.0; }

void orc_model_set_params(orc_model *m, const double *k, const double *c)
{
    if (k) memcpy(m->k, k, sizeof(double) * (size_t)m->S);
    if (c) memcpy(m->c, c, sizeof(double) * (size_t)m->S);
}

void orc_model_free(orc_model *m)
{
    if (!m) return;
    free(m->w); free(m->ends); free(m->rest); free(m->k); free(m->c);
    free(m->verts); free(m->tris); free(m->tA); free(m->tn); free(m->tlo); free(m->thi);
    free(m->cell_start); free(m->cell_tris); free(m->fext);
    free(m);
}

/* ------------------------------------------------------------------ 1. spring forces */

/* F[N][3] = sum of Alg. 1 spring forces at state (x, v). */
void orc_forces(const orc_model *m, const double *x, const double *v, double *F)
{
    memset(F, 0, sizeof(double) * 3 * (size_t)m->N);
    for (int s = 0; s < m->S; ++s) {
        int a = m->ends[2 * s], b = m->ends[2 * s + 1];
        double d[3], dir[3];
        sub3(x + 3 * b, x + 3 * a, d);
        double len = sqrt(dot3(d, d));
        for (int q = 0; q < 3; ++q) dir[q] = d[q] / len;
        double spring = m->k[s] * (len - m->rest[s]);
        double damp = m->c[s] * (dot3(v + 3 * b, dir) - dot3(v + 3 * a, dir));
        for (int q = 0; q < 3; ++q) {
            double f = (spring + damp) * dir[q];
            F[3 * a + q] += f;
            F[3 * b + q] -= f;
        }
    }
}

/* ------------------------------------------------------------------ point-triangle distance */

/* Squared distance from p to the closed segment [a, b]. */
static double seg_dist2(const double *p, const double *a, const double *b)
{
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double L2 = dot3(ab, ab);
    double t = L2 > 0 ? dot3(ap, ab) / L2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double r[3];
    for (int q = 0; q < 3; ++q) r[q] = ap[q] - t * ab[q];
    return dot3(r, r);
}

/* Squared distance from p to the closed triangle (A, B, C): the distance to the plane if
 * p's orthogonal projection lies inside the triangle, otherwise the distance to the
 * nearest of the three edges. */
double orc_point_tri_dist2(const double *p, const double *A, const double *B, const double *C)
{
    double e1[3], e2[3], n[3], ap[3];
    sub3(B, A, e1);
    sub3(C, A, e2);
    cross3(e1, e2, n);
    double nn = dot3(n, n);
    sub3(p, A, ap);
    double sd = dot3(ap, n);
    /* projection q = p - (sd/nn) n; barycentric signs from sub-triangle orientations */
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = p[i] - sd / nn * n[i];
    double t0[3], t1[3], c0[3], c1[3], c2[3];
    sub3(B, q, t0); sub3(C, q, t1); cross3(t0, t1, c0); /* opposite A */
    sub3(C, q, t0); sub3(A, q, t1); cross3(t0, t1, c1); /* opposite B */
    sub3(A, q, t0); sub3(B, q, t1); cross3(t0, t1, c2); /* opposite C */
    if (dot3(c0, n) >= 0 && dot3(c1, n) >= 0 && dot3(c2, n) >= 0) return sd * sd / nn;
    double d0 = seg_dist2(p, A, B), d1 = seg_dist2(p, B, C), d2 = seg_dist2(p, C, A);
    double d = d0 < d1 ? d0 : d1;
    return d < d2 ? d : d2;
}

/* ------------------------------------------------------------------ one substep */

static int in_box(const orc_model *m, int t, const double *p)
{
    for (int a = 0; a < 3; ++a)
        if (p[a] < m->tlo[3 * t + a] || p[a] > m->thi[3 * t + a]) return 0;
    return 1;
}

/* Contacts of point p: triangles with dist(p, t) < th, in ascending triangle id.
 * Writes up to cap ids into out and returns the count; *margin (if given) receives the
 * smallest |dist - th| over every triangle whose (slack-inflated) box holds p. */
static int contacts_of(const orc_model *m, const double *p, int *out, int cap, double *margin)
{
    if (m->T == 0) { if (margin) *margin = INFINITY; return 0; }
    int ci = cell_coord(m, p[0], 0), cj = cell_coord(m, p[1], 1), ck = cell_coord(m, p[2], 2);
    long long id = ((long long)ck * m->dim[1] + cj) * m->dim[0] + ci;
    int n = 0;
    double mg = INFINITY;
    for (int r = m->cell_start[id]; r < m->cell_start[id + 1]; ++r) {
        int t = m->cell_tris[r];
        if (!in_box(m, t, p)) continue;
        const double *A = m->verts + 3 * m->tris[3 * t];
        const double *B = m->verts + 3 * m->tris[3 * t + 1];
        const double *C = m->verts + 3 * m->tris[3 * t + 2];
        double d = sqrt(orc_point_tri_dist2(p, A, B, C));
        double gap = fabs(d - m->th);
        if (gap < mg) mg = gap;
        if (d < m->th) {
            if (n < cap) out[n] = t;
            ++n;
        }
    }
    if (margin) *margin = mg;
    return n;
}

#define ORC_MAX_CONTACTS 512

/* Forces and integration of one substep without collision: (x, v) -> (x*, v*) in place. */
void orc_predict(const orc_model *m, double *x, double *v, double h)
{
    int N = m->N;
    double *F = malloc(sizeof(double) * 3 * (size_t)N);
    orc_forces(m, x, v, F);
    for (int i = 0; i < N; ++i) {
        if (m->w[i] == 0.0) {
            for (int q = 0; q < 3; ++q) v[3 * i + q] = 0.0;
            continue;
        }
        for (int q = 0; q < 3; ++q) {
            v[3 * i + q] = v[3 * i + q] + h * (m->w[i] * (F[3 * i + q] + fext_of(m, i, q)) + m->g[q]);
            x[3 * i + q] = x[3 * i + q] + h * v[3 * i + q];
        }
    }
    free(F);
}

/* Response of one node at predicted (p, v) to the contact triangles ids[0..n) (ascending):
 * p <- p + mean_t (th - (p - A_t).n_t) n_t, v <- -restitution v; unchanged if n == 0. */
void orc_respond(const orc_model *m, double *p, double *v, const int *ids, int n)
{
    if (n <= 0) return;
    double sum[3] = {0, 0, 0};
    for (int r = 0; r < n; ++r) {
        int t = ids[r];
        const double *nt = m->tn + 3 * t;
        double ap[3];
        sub3(p, m->tA + 3 * t, ap);
        double push = m->th - dot3(ap, nt);
        for (int q = 0; q < 3; ++q) sum[q] += push * nt[q];
    }
    for (int q = 0; q < 3; ++q) {
        p[q] = p[q] + sum[q] / n;
        v[q] = -m->restitution * v[q];
    }
}

/* Every triangle whose slack-inflated box holds p, ascending, with its exact distance to p.
 * Returns the count (entries beyond cap are counted, not written). */
int orc_box_candidates(const orc_model *m, const double *p, int *ids, double *dist, int cap)
{
    if (m->T == 0) return 0;
    int ci = cell_coord(m, p[0], 0), cj = cell_coord(m, p[1], 1), ck = cell_coord(m, p[2], 2);
    long long id = ((long long)ck * m->dim[1] + cj) * m->dim[0] + ci;
    int n = 0;
    for (int r = m->cell_start[id]; r < m->cell_start[id + 1]; ++r) {
        int t = m->cell_tris[r];
        if (!in_box(m, t, p)) continue;
        if (n < cap) {
            ids[n] = t;
            dist[n] = sqrt(orc_point_tri_dist2(p, m->verts + 3 * m->tris[3 * t],
                                               m->verts + 3 * m->tris[3 * t + 1],
                                               m->verts + 3 * m->tris[3 * t + 2]));
        }
        ++n;
    }
    return n;
}

/* Advance (x, v) [N][3] by one substep of length h, in place.
 * count (optional, [N]) receives each node's number of contacts; margin (optional, [N])
 * the smallest |dist - th| over its box candidates (INFINITY if none). */
void orc_substep(const orc_model *m, double *x, double *v, double h, int *count, double *margin)
{
    int N = m->N;
    orc_predict(m, x, v, h);
    int ids[ORC_MAX_CONTACTS];
    for (int i = 0; i < N; ++i) {
        if (count) count[i] = 0;
        if (margin) margin[i] = INFINITY;
        if (m->w[i] == 0.0) continue;
        int n = contacts_of(m, x + 3 * i, ids, ORC_MAX_CONTACTS, margin ? margin + i : NULL);
        if (count) count[i] = n;
        if (n > ORC_MAX_CONTACTS) n = ORC_MAX_CONTACTS;
        orc_respond(m, x + 3 * i, v + 3 * i, ids, n);
    }
}

/* n_sub substeps in sequence. */
void orc_run(const orc_model *m, double *x, double *v, double h, int n_sub)
{
    for (int s = 0; s < n_sub; ++s) orc_substep(m, x, v, h, NULL, NULL);
}

/* One substep with the contact sets held fixed: the prediction of orc_predict, then node
 * i's response to the triangles ids[off[i] .. off[i+1]) (ascending), whatever their
 * distance to the prediction.  With the sets orc_substep finds this is orc_substep; with
 * any fixed sets it is one smooth piece of the step, the function whose derivative the
 * adjoint computes (contact set frozen). */
void orc_substep_given(const orc_model *m, double *x, double *v, double h, const int *off,
                       const int *ids)
{
    orc_predict(m, x, v, h);
    for (int i = 0; i < m->N; ++i) {
        if (m->w[i] == 0.0) continue; /* pinned nodes never collide */
        orc_respond(m, x + 3 * i, v + 3 * i, ids + off[i], off[i + 1] - off[i]);
    }
}

/* n_sub substeps of orc_substep_given; substep s uses the sets off[s*(N+1) + i] ..
 * off[s*(N+1) + i + 1] of ids (offsets into the one ids array). */
void orc_run_given(const orc_model *m, double *x, double *v, double h, int n_sub,
                   const int *off, const int *ids)
{
    for (int s = 0; s < n_sub; ++s)
        orc_substep_given(m, x, v, h, off + (size_t)s * (m->N + 1), ids);
}

/* Checks another implementation's contact sets against the distances at the predicted
 * positions xp: node i's set ids[off[i] .. off[i+1]) is valid iff it holds every triangle
 * within th - border of xp_i and only triangles within th + border (a decision closer than
 * border to the threshold may go either way in lower precision), and a pinned node has
 * none.  status[i] = 0 valid, 1 a listed triangle is too far, 2 a sure contact is missing,
 * 3 a pinned node has contacts.  Returns the number of invalid nodes; *n_border (optional)
 * receives the number of listed triangles whose distance lies within border of th. */
int orc_check_contacts(const orc_model *m, const double *xp, double border, const int *off,
                       const int *ids, int *status, long long *n_border)
{
    int bad = 0;
    long long nb = 0;
    int sure[ORC_MAX_CONTACTS];
    for (int i = 0; i < m->N; ++i) {
        const double *p = xp + 3 * i;
        int st = 0, n = off[i + 1] - off[i];
        if (m->w[i] == 0.0) {
            if (n > 0) st = 3;
        } else {
            for (int r = 0; r < n && !st; ++r) {
                int t = ids[off[i] + r];
                if (t < 0 || t >= m->T) { st = 1; break; }
                double d = sqrt(orc_point_tri_dist2(p, m->verts + 3 * m->tris[3 * t],
                                                    m->verts + 3 * m->tris[3 * t + 1],
                                                    m->verts + 3 * m->tris[3 * t + 2]));
                if (d >= m->th + border) st = 1;
                else if (d >= m->th - border) ++nb;
            }
            if (!st && m->T > 0) {
                /* the triangles within th - border are among those within th */
                int ns = contacts_of(m, p, sure, ORC_MAX_CONTACTS, NULL);
                if (ns > ORC_MAX_CONTACTS) ns = ORC_MAX_CONTACTS;
                for (int a = 0; a < ns && !st; ++a) {
                    int t = sure[a];
                    double d = sqrt(orc_point_tri_dist2(p, m->verts + 3 * m->tris[3 * t],
                                                        m->verts + 3 * m->tris[3 * t + 1],
                                                        m->verts + 3 * m->tris[3 * t + 2]));
                    if (d >= m->th - border) continue;
                    int found = 0;
                    for (int r = 0; r < n; ++r) found |= ids[off[i] + r] == t;
                    if (!found) st = 2;
                }
            }
        }
        if (status) status[i] = st;
        bad += st != 0;
    }
    if (n_border) *n_border = nb;
    return bad;
}

/* Number of contacts a node at p would get, and the contact triangle ids (ascending). */
int orc_contacts(const orc_model *m, const double *p, int *out, int cap)
{
    return contacts_of(m, p, out, cap, NULL);
}

/* ------------------------------------------------------------------ FP32 broad-phase predicate */

/* Brute force over all (node, triangle) pairs in FP32: node i is a candidate of triangle t
 * iff lo_t <= x_i <= hi_t on every axis, where lo_t = fl32(min of t's vertex coordinates -
 * th) and hi_t = fl32(max + th).  Pinned-ness is ignored here.  Pairs are written as
 * (node, tri) in ascending node, then triangle, order; returns the total pair count (pairs
 * beyond cap are counted but not written). */
long long orc_candidates_f32(int N, const float *x, int T, const float *verts, const int *tris,
                             float th, int *pairs, long long cap)
{
    float *lo = malloc(sizeof(float) * 3 * (size_t)(T + 1));
    float *hi = malloc(sizeof(float) * 3 * (size_t)(T + 1));
    for (int t = 0; t < T; ++t) {
        for (int a = 0; a < 3; ++a) {
            float va = verts[3 * tris[3 * t] + a], vb = verts[3 * tris[3 * t + 1] + a],
                  vc = verts[3 * tris[3 * t + 2] + a];
            float mn = va < vb ? va : vb;
            mn = mn < vc ? mn : vc;
            float mx = va > vb ? va : vb;
            mx = mx > vc ? mx : vc;
            lo[3 * t + a] = mn - th;
            hi[3 * t + a] = mx + th;
        }
    }
    long long n = 0;
    for (int i = 0; i < N; ++i) {
        const float *p = x + 3 * i;
        for (int t = 0; t < T; ++t) {
            int in = 1;
            for (int a = 0; a < 3; ++a)
                if (!(lo[3 * t + a] <= p[a] && p[a] <= hi[3 * t + a])) { in = 0; break; }
            if (in) {
                if (n < cap) { pairs[2 * n] = i; pairs[2 * n + 1] = t; }
                ++n;
            }
        }
    }
    free(lo);
    free(hi);
    return n;
}

/* ------------------------------------------------------------------ adjoint of one substep */

/* Reverse-mode derivative of orc_substep at state (x, v) with the contact set held fixed.
 * Given xb_out, vb_out = dL/d(x, v) after the substep, writes xb_in, vb_in = dL/d(x, v)
 * before it and ADDS dL/dk, dL/dc into kb, cb (either may be NULL).  The contact sets are
 * those orc_substep finds at the prediction; the transpose itself is orc_substep_vjp_given. */
void orc_substep_vjp_given(const orc_model *m, const double *x, const double *v, double h,
                           const int *off, const int *ids, const double *xb_out,
                           const double *vb_out, double *xb_in, double *vb_in, double *kb,
                           double *cb);

void orc_substep_vjp(const orc_model *m, const double *x, const double *v, double h,
                     const double *xb_out, const double *vb_out, double *xb_in, double *vb_in,
                     double *kb, double *cb)
{
    int N = m->N;
    double *xp = malloc(sizeof(double) * 3 * (size_t)N);
    double *vp = malloc(sizeof(double) * 3 * (size_t)N);
    int *off = malloc(sizeof(int) * ((size_t)N + 1));
    size_t cap = 4 * (size_t)N + 16, len = 0;
    int *ids = malloc(sizeof(int) * cap);
    memcpy(xp, x, sizeof(double) * 3 * (size_t)N);
    memcpy(vp, v, sizeof(double) * 3 * (size_t)N);
    orc_predict(m, xp, vp, h);
    int buf[ORC_MAX_CONTACTS];
    off[0] = 0;
    for (int i = 0; i < N; ++i) {
        int n = 0;
        if (m->w[i] != 0.0) {
            n = contacts_of(m, xp + 3 * i, buf, ORC_MAX_CONTACTS, NULL);
            if (n > ORC_MAX_CONTACTS) n = ORC_MAX_CONTACTS;
        }
        if (len + (size_t)n > cap) {
            cap = 2 * (len + (size_t)n);
            ids = realloc(ids, sizeof(int) * cap);
        }
        memcpy(ids + len, buf, sizeof(int) * (size_t)n);
        len += (size_t)n;
        off[i + 1] = (int)len;
    }
    orc_substep_vjp_given(m, x, v, h, off, ids, xb_out, vb_out, xb_in, vb_in, kb, cb);
    free(xp);
    free(vp);
    free(off);
    free(ids);
}

/* Reverse-mode derivative of orc_substep_given (the substep with node i's contact
 * triangles ids[off[i] .. off[i+1]), ascending, held fixed):
 *   response  x' = x* + mean_t (th - (x* - A_t).n_t) n_t, so dx'/dx* = I - mean_t n_t n_t^T,
 *             and v' = -r v*, so dv'/dv* = -r I (identity for a node without contacts);
 *   integration x* = x + h v*, v* = v + h (w F + g);
 *   spring forces transposed spring by spring. */
void orc_substep_vjp_given(const orc_model *m, const double *x, const double *v, double h,
                           const int *off, const int *ids, const double *xb_out,
                           const double *vb_out, double *xb_in, double *vb_in, double *kb,
                           double *cb)
{
    int N = m->N;
    double *F = malloc(sizeof(double) * 3 * (size_t)N);
    double *Fb = calloc(3 * (size_t)N, sizeof(double));
    orc_forces(m, x, v, F);
    for (int i = 0; i < N; ++i) {
        if (m->w[i] == 0.0) {
            for (int q = 0; q < 3; ++q) { xb_in[3 * i + q] = xb_out[3 * i + q]; vb_in[3 * i + q] = 0.0; }
            continue;
        }
        int n = off[i + 1] - off[i];
        double xbs[3], vbs[3];
        for (int q = 0; q < 3; ++q) { xbs[q] = xb_out[3 * i + q]; vbs[q] = vb_out[3 * i + q]; }
        if (n > 0) {
            double acc[3] = {0, 0, 0};
            for (int r = 0; r < n; ++r) {
                const double *nt = m->tn + 3 * ids[off[i] + r];
                double s = dot3(nt, xbs);
                for (int q = 0; q < 3; ++q) acc[q] += s * nt[q];
            }
            for (int q = 0; q < 3; ++q) {
                xbs[q] = xbs[q] - acc[q] / n;
                vbs[q] = -m->restitution * vbs[q];
            }
        }
        for (int q = 0; q < 3; ++q) {
            double vtot = vbs[q] + h * xbs[q];
            xb_in[3 * i + q] = xbs[q];
            vb_in[3 * i + q] = vtot;
            Fb[3 * i + q] = h * m->w[i] * vtot;
        }
    }
    for (int s = 0; s < m->S; ++s) {
        int a = m->ends[2 * s], b = m->ends[2 * s + 1];
        double d[3], u[3], dv[3], lam[3];
        sub3(x + 3 * b, x + 3 * a, d);
        sub3(v + 3 * b, v + 3 * a, dv);
        sub3(Fb + 3 * a, Fb + 3 * b, lam);
        double len = sqrt(dot3(d, d));
        for (int q = 0; q < 3; ++q) u[q] = d[q] / len;
        double dvu = dot3(dv, u);
        double phi = m->k[s] * (len - m->rest[s]) + m->c[s] * dvu;
        double ul = dot3(u, lam);
        double db[3], dvb[3];
        for (int q = 0; q < 3; ++q) {
            double perp_l = lam[q] - u[q] * ul;
            double perp_dv = dv[q] - u[q] * dvu;
            db[q] = phi / len * perp_l + m->k[s] * u[q] * ul + m->c[s] / len * perp_dv * ul;
            dvb[q] = m->c[s] * u[q] * ul;
        }
        for (int q = 0; q < 3; ++q) {
            xb_in[3 * b + q] += db[q];
            xb_in[3 * a + q] -= db[q];
            vb_in[3 * b + q] += dvb[q];
            vb_in[3 * a + q] -= dvb[q];
        }
        if (kb) kb[s] += (len - m->rest[s]) * ul;
        if (cb) cb[s] += dvu * ul;
    }
    free(F);
    free(Fb);
}

/* ------------------------------------------------------------------ rollout gradient */

/* Run n_sub substeps from (x0, v0) and back-propagate.
 *   out_sub[j] (ascending, 1..n_sub): substep counts after which the loss reads x;
 *   xbar[j][N][3]: dL/dx at those states.
 * Writes x_out[j][N][3] (the states themselves, if x_out is not NULL) and the gradients
 * gk[S], gc[S], gv0[N][3], gx0[N][3] (any may be NULL).  States are checkpointed every
 * ckpt substeps (ckpt >= 1) and each segment is recomputed from its checkpoint on the way
 * back; the values do not depend on ckpt. */
void orc_rollout_grad(const orc_model *m, const double *x0, const double *v0, double h,
                      int n_sub, int n_out, const int *out_sub, const double *xbar,
                      int ckpt, double *x_out, double *gk, double *gc, double *gv0,
                      double *gx0)
{
    int N = m->N, S = m->S;
    size_t n3 = 3 * (size_t)N;
    if (ckpt < 1) ckpt = 1;
    int n_ck = n_sub / ckpt + 1;
    double *ck_x = malloc(sizeof(double) * n3 * (size_t)n_ck);
    double *ck_v = malloc(sizeof(double) * n3 * (size_t)n_ck);
    double *x = malloc(sizeof(double) * n3), *v = malloc(sizeof(double) * n3);
    memcpy(x, x0, sizeof(double) * n3);
    memcpy(v, v0, sizeof(double) * n3);
    int j = 0;
    for (int s = 0; s <= n_sub; ++s) {
        if (s % ckpt == 0) {
            memcpy(ck_x + n3 * (size_t)(s / ckpt), x, sizeof(double) * n3);
            memcpy(ck_v + n3 * (size_t)(s / ckpt), v, sizeof(double) * n3);
        }
        while (j < n_out && out_sub[j] == s) {
            if (x_out) memcpy(x_out + n3 * (size_t)j, x, sizeof(double) * n3);
            ++j;
        }
        if (s < n_sub) orc_substep(m, x, v, h, NULL, NULL);
    }
    double *kb = calloc((size_t)S + 1, sizeof(double)), *cb = calloc((size_t)S + 1, sizeof(double));
    double *xb = calloc(n3, sizeof(double)), *vb = calloc(n3, sizeof(double));
    double *xb2 = malloc(sizeof(double) * n3), *vb2 = malloc(sizeof(double) * n3);
    double *seg_x = malloc(sizeof(double) * n3 * (size_t)ckpt);
    double *seg_v = malloc(sizeof(double) * n3 * (size_t)ckpt);
    /* backward, one checkpoint segment at a time: recompute the segment's states from its
     * checkpoint, then apply the substep adjoints in reverse order */
    j = n_out - 1;
    while (j >= 0 && out_sub[j] == n_sub) {
        for (size_t q = 0; q < n3; ++q) xb[q] += xbar[n3 * (size_t)j + q];
        --j;
    }
    for (int seg = (n_sub - 1) / ckpt; seg >= 0 && n_sub > 0; --seg) {
        int base = seg * ckpt;
        int top = base + ckpt < n_sub ? base + ckpt : n_sub; /* substeps base..top-1 */
        memcpy(seg_x, ck_x + n3 * (size_t)seg, sizeof(double) * n3);
        memcpy(seg_v, ck_v + n3 * (size_t)seg, sizeof(double) * n3);
        for (int r = 1; r < top - base; ++r) {
            memcpy(seg_x + n3 * (size_t)r, seg_x + n3 * (size_t)(r - 1), sizeof(double) * n3);
            memcpy(seg_v + n3 * (size_t)r, seg_v + n3 * (size_t)(r - 1), sizeof(double) * n3);
            orc_substep(m, seg_x + n3 * (size_t)r, seg_v + n3 * (size_t)r, h, NULL, NULL);
        }
        for (int s = top; s > base; --s) {
            int slot = s - 1 - base; /* state before substep s-1 -> s */
            orc_substep_vjp(m, seg_x + n3 * (size_t)slot, seg_v + n3 * (size_t)slot, h, xb, vb,
                            xb2, vb2, kb, cb);
            memcpy(xb, xb2, sizeof(double) * n3);
            memcpy(vb, vb2, sizeof(double) * n3);
            while (j >= 0 && out_sub[j] == s - 1) {
                for (size_t q = 0; q < n3; ++q) xb[q] += xbar[n3 * (size_t)j + q];
                --j;
            }
        }
    }
    if (gk) memcpy(gk, kb, sizeof(double) * (size_t)S);
    if (gc) memcpy(gc, cb, sizeof(double) * (size_t)S);
    if (gv0) memcpy(gv0, vb, sizeof(double) * n3);
    if (gx0) memcpy(gx0, xb, sizeof(double) * n3);
    free(ck_x); free(ck_v); free(x); free(v); free(kb); free(cb);
    free(xb); free(vb); free(xb2); free(vb2); free(seg_x); free(seg_v);
}

/* ------------------------------------------------------------------ extended Moller-Trumbore narrow phase */

/* Segment S -> E against triangle (V0, V1, V2), following the steps of Sec. 3's extended
 * Moller-Trumbore process: with d = E - S and r = d / |d|, e1 = V1 - V0, e2 = V2 - V0,
 * h = r x e2 and a = e1 . h, the segment is parallel when |a| < eps; otherwise with
 * f = 1 / a, s = S - V0: u = f (s . h) must lie in [0, 1], and with q = s x e1,
 * v = f (r . q) >= 0, u + v <= 1 and t = f (e2 . q) strictly inside (eps, |d|).  Returns 1
 * for a crossing (then *t_out = t, the distance from S to the crossing point S + t r).
 * A zero-length segment crosses nothing.  *margin (optional) receives the smallest distance,
 * in metres, of the decision quantities from their bounds (u, 1 - u, v, 1 - u - v scaled by
 * the longer triangle edge; t - eps and |d| - t), INFINITY when parallel or degenerate. */
int orc_mt(const double *S, const double *E, const double *V0, const double *V1,
           const double *V2, double eps, double *t_out, double *margin)
{
    if (margin) *margin = INFINITY;
    double d[3], r[3], e1[3], e2[3], h[3], sv[3], q[3];
    sub3(E, S, d);
    double len = sqrt(dot3(d, d));
    if (!(len > 0.0)) return 0;
    for (int k = 0; k < 3; ++k) r[k] = d[k] / len;
    sub3(V1, V0, e1);
    sub3(V2, V0, e2);
    cross3(r, e2, h);
    double a = dot3(e1, h);
    if (fabs(a) < eps) return 0;
    double f = 1.0 / a;
    sub3(S, V0, sv);
    double u = f * dot3(sv, h);
    cross3(sv, e1, q);
    double v = f * dot3(r, q);
    double t = f * dot3(e2, q);
    if (margin) {
        double L = fmax(sqrt(dot3(e1, e1)), sqrt(dot3(e2, e2)));
        double m = fmin(fmin(fabs(u), fabs(1.0 - u)), fmin(fabs(v), fabs(1.0 - u - v))) * L;
        m = fmin(m, fmin(fabs(t - eps), fabs(len - t)));
        *margin = m;
    }
    if (u < 0.0 || u > 1.0) return 0;
    if (v < 0.0 || u + v > 1.0) return 0;
    if (!(eps < t && t < len)) return 0;
    if (t_out) *t_out = t;
    return 1;
}

/* Triangles of the cloth grid that contain node i = (row, col): each quad (r, c), (r+1, c),
 * (r+1, c+1), (r, c+1) is split along its (r, c)-(r+1, c+1) diagonal into (a, b, c) and
 * (a, c, d).  Writes up to 6 triangles (vertex triples) and returns their count. */
static int cloth_tris_of(int nx, int ny, int i, int tri[6][3])
{
    int row = i / nx, col = i % nx, n = 0;
    for (int qr = row - 1; qr <= row; ++qr)
        for (int qc = col - 1; qc <= col; ++qc) {
            if (qr < 0 || qc < 0 || qr + 1 >= ny || qc + 1 >= nx) continue;
            int a = qr * nx + qc, b = (qr + 1) * nx + qc, c = (qr + 1) * nx + qc + 1, d = qr * nx + qc + 1;
            int two[2][3] = {{a, b, c}, {a, c, d}};
            for (int k = 0; k < 2; ++k)
                if (two[k][0] == i || two[k][1] == i || two[k][2] == i) {
                    for (int z = 0; z < 3; ++z) tri[n][z] = two[k][z];
                    ++n;
                }
        }
    return n;
}

/* Cloth-mesh edges at node i (the triangles' edges: grid neighbours along rows and columns
 * and the split diagonal), as neighbour ids.  Returns their count (at most 6). */
static int cloth_edges_of(int nx, int ny, int i, int nb[6])
{
    int row = i / nx, col = i % nx, n = 0;
    int dr[6] = {0, 0, 1, -1, 1, -1}, dc[6] = {1, -1, 0, 0, 1, -1};
    for (int k = 0; k < 6; ++k) {
        int r2 = row + dr[k], c2 = col + dc[k];
        if (r2 < 0 || c2 < 0 || r2 >= ny || c2 >= nx) continue;
        nb[n++] = r2 * nx + c2;
    }
    return n;
}

static void aabb_add(double lo[3], double hi[3], const double *p)
{
    for (int a = 0; a < 3; ++a) {
        if (p[a] < lo[a]) lo[a] = p[a];
        if (p[a] > hi[a]) hi[a] = p[a];
    }
}

static int box_overlaps(const orc_model *m, int t, const double lo[3], const double hi[3])
{
    for (int a = 0; a < 3; ++a)
        if (hi[a] < m->tlo[3 * t + a] || lo[a] > m->thi[3 * t + a]) return 0;
    return 1;
}

#define ORC_MT_EPS 1e-7

/* The contact set of node i under the triangle-triangle narrow phase (Sec. 3): surface
 * triangle t is a contact of i when
 *   (A) a cloth edge at i, at predicted positions xp, crosses t (oriented from the lower
 *       node id), or
 *   (B) an edge of t (oriented from the lower vertex id) crosses a cloth triangle at i, at xp
 *       (so every triangle next to a surface edge that pierces the cloth is a contact of
 *       that cloth triangle's three nodes), or
 *   (C) i's own path from xs to xp crosses t (the continuous test).
 * Pinned nodes have no contacts.  Candidates are the triangles whose slack-inflated box
 * overlaps the box of i's edges, cloth triangles and path; a crossing point lies in both
 * boxes, so the filter never changes the result.  Writes up to cap ids in ascending order and
 * returns the count; *margin receives the smallest decision margin over every test made. */
/* Whether node i's tests (A), (B), (C) find a crossing with triangle t; *mg receives the
 * smallest decision margin over those tests. */
static int mt_pair(const orc_model *m, const double *xs, const double *xp, int i, int t,
                   const int *nb, int nnb, int tri[6][3], int ntri, double *mg)
{
    const int *tv = m->tris + 3 * t;
    const double *V0 = m->verts + 3 * tv[0], *V1 = m->verts + 3 * tv[1], *V2 = m->verts + 3 * tv[2];
    int hit = 0;
    double g, best = INFINITY;
    for (int k = 0; k < nnb; ++k) {            /* (A) */
        int p0 = i < nb[k] ? i : nb[k], p1 = i < nb[k] ? nb[k] : i;
        hit |= orc_mt(xp + 3 * p0, xp + 3 * p1, V0, V1, V2, ORC_MT_EPS, NULL, &g);
        if (g < best) best = g;
    }
    for (int k = 0; k < ntri; ++k)             /* (B) */
        for (int z = 0; z < 3; ++z) {
            int u0 = tv[z], u1 = tv[(z + 1) % 3];
            int w0 = u0 < u1 ? u0 : u1, w1 = u0 < u1 ? u1 : u0;
            hit |= orc_mt(m->verts + 3 * w0, m->verts + 3 * w1, xp + 3 * tri[k][0],
                          xp + 3 * tri[k][1], xp + 3 * tri[k][2], ORC_MT_EPS, NULL, &g);
            if (g < best) best = g;
        }
    hit |= orc_mt(xs + 3 * i, xp + 3 * i, V0, V1, V2, ORC_MT_EPS, NULL, &g);  /* (C) */
    if (g < best) best = g;
    *mg = best;
    return hit;
}

/* Every candidate triangle of node i (ascending id) with whether it is a contact and the
 * smallest decision margin of its tests.  Returns the candidate count (entries beyond cap
 * are counted, not written).  Candidates are the triangles whose slack-inflated box
 * overlaps the box of i's path, edges and cloth triangles. */
int orc_mt_candidates(const orc_model *m, int nx, int ny, const double *xs, const double *xp,
                      int i, int *ids, int *hits, double *margins, int cap)
{
    if (m->T == 0 || m->w[i] == 0.0) return 0;
    int tri[6][3], nb[6];
    int ntri = cloth_tris_of(nx, ny, i, tri), nnb = cloth_edges_of(nx, ny, i, nb);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    aabb_add(lo, hi, xs + 3 * i);
    aabb_add(lo, hi, xp + 3 * i);
    for (int k = 0; k < nnb; ++k) aabb_add(lo, hi, xp + 3 * nb[k]);
    int clo[3], chi[3];
    for (int a = 0; a < 3; ++a) { clo[a] = cell_coord(m, lo[a], a); chi[a] = cell_coord(m, hi[a], a); }
    char *seen = calloc((size_t)m->T, 1);
    for (int ck = clo[2]; ck <= chi[2]; ++ck)
        for (int cj = clo[1]; cj <= chi[1]; ++cj)
            for (int ci = clo[0]; ci <= chi[0]; ++ci) {
                long long id = ((long long)ck * m->dim[1] + cj) * m->dim[0] + ci;
                for (int r = m->cell_start[id]; r < m->cell_start[id + 1]; ++r) {
                    int t = m->cell_tris[r];
                    if (!seen[t] && box_overlaps(m, t, lo, hi)) seen[t] = 1;
                }
            }
    int n = 0;
    for (int t = 0; t < m->T; ++t) {
        if (!seen[t]) continue;
        double mg;
        int hit = mt_pair(m, xs, xp, i, t, nb, nnb, tri, ntri, &mg);
        if (n < cap) { ids[n] = t; hits[n] = hit; margins[n] = mg; }
        ++n;
    }
    free(seen);
    return n;
}

/* The contact set of node i under the triangle-triangle narrow phase (Sec. 3): surface
 * triangle t is a contact of i when
 *   (A) a cloth edge at i, at predicted positions xp, crosses t (oriented from the lower
 *       node id), or
 *   (B) an edge of t (oriented from the lower vertex id) crosses a cloth triangle at i, at xp
 *       (so every triangle next to a surface edge that pierces the cloth is a contact of
 *       that cloth triangle's three nodes), or
 *   (C) i's own path from xs to xp crosses t (the continuous test).
 * Pinned nodes have no contacts.  Candidates are the triangles whose slack-inflated box
 * overlaps the box of i's edges, cloth triangles and path; a crossing point lies in both
 * boxes, so the filter never changes the result.  Writes up to cap ids in ascending order and
 * returns the count; *margin receives the smallest decision margin over every test made. */
int orc_mt_contacts(const orc_model *m, int nx, int ny, const double *xs, const double *xp,
                    int i, int *out, int cap, double *margin)
{
    int ncand = orc_mt_candidates(m, nx, ny, xs, xp, i, NULL, NULL, NULL, 0);
    int *ids = malloc(sizeof(int) * (size_t)(ncand + 1)), *hits = malloc(sizeof(int) * (size_t)(ncand + 1));
    double *mgs = malloc(sizeof(double) * (size_t)(ncand + 1));
    orc_mt_candidates(m, nx, ny, xs, xp, i, ids, hits, mgs, ncand);
    double mg = INFINITY;
    int n = 0;
    for (int r = 0; r < ncand; ++r) {
        if (mgs[r] < mg) mg = mgs[r];
        if (hits[r]) {
            if (n < cap) out[n] = ids[r];
            ++n;
        }
    }
    free(ids); free(hits); free(mgs);
    if (margin) *margin = mg;
    return n;
}

/* One substep with the triangle-triangle narrow phase: prediction as in orc_substep, every
 * node's contact set from the start positions and the predictions of all nodes, then the
 * averaged response of each node (x* + mean (th - s_t) n_t, v <- -restitution v*). */
void orc_substep_mt(const orc_model *m, int nx, int ny, double *x, double *v, double h,
                    int *count, double *margin)
{
    int N = m->N;
    double *xs = malloc(sizeof(double) * 3 * (size_t)N);
    memcpy(xs, x, sizeof(double) * 3 * (size_t)N);
    orc_predict(m, x, v, h);
    double *xp = malloc(sizeof(double) * 3 * (size_t)N);
    memcpy(xp, x, sizeof(double) * 3 * (size_t)N);
    int ids[ORC_MAX_CONTACTS];
    for (int i = 0; i < N; ++i) {
        double mg;
        int n = orc_mt_contacts(m, nx, ny, xs, xp, i, ids, ORC_MAX_CONTACTS, &mg);
        if (count) count[i] = n;
        if (margin) margin[i] = mg;
        if (n > ORC_MAX_CONTACTS) n = ORC_MAX_CONTACTS;
        orc_respond(m, x + 3 * i, v + 3 * i, ids, n);
    }
    free(xs);
    free(xp);
}

/* ------------------------------------------------------------------ vertex normals */

/* Per-vertex normals of an nx-by-ny cloth grid (node (i, j) = i*nx + j, Sec. 3's normal
 * update before rendering): each quad (i, j)-(i+1, j)-(i+1, j+1)-(i, j+1) is split into the
 * triangles (a, b, c) and (a, c, d) along its (i, j)-(i+1, j+1) diagonal; every triangle adds
 * its cross product (B - A) x (C - A) -- twice its area times its unit normal -- to its three
 * vertices, and each vertex sum is normalised (a zero sum stays zero). */
void orc_vertex_normals(int nx, int ny, const double *x, double *n)
{
    memset(n, 0, sizeof(double) * 3 * (size_t)nx * (size_t)ny);
    for (int i = 0; i + 1 < ny; ++i)
        for (int j = 0; j + 1 < nx; ++j) {
            int a = i * nx + j, b = (i + 1) * nx + j, c = (i + 1) * nx + j + 1, d = i * nx + j + 1;
            int tri[2][3] = {{a, b, c}, {a, c, d}};
            for (int t = 0; t < 2; ++t) {
                double e1[3], e2[3], cr[3];
                sub3(x + 3 * tri[t][1], x + 3 * tri[t][0], e1);
                sub3(x + 3 * tri[t][2], x + 3 * tri[t][0], e2);
                cross3(e1, e2, cr);
                for (int k = 0; k < 3; ++k)
                    for (int q = 0; q < 3; ++q) n[3 * tri[t][k] + q] += cr[q];
            }
        }
    for (long long v = 0; v < (long long)nx * ny; ++v) {
        double len = sqrt(dot3(n + 3 * v, n + 3 * v));
        if (len > 0)
            for (int q = 0; q < 3; ++q) n[3 * v + q] /= len;
    }
}

/* ------------------------------------------------------------------ accessors */

void orc_model_triangle(const orc_model *m, int t, double *A, double *n, double *lo, double *hi)
{
    for (int a = 0; a < 3; ++a) {
        if (A) A[a] = m->tA[3 * t + a];
        if (n) n[a] = m->tn[3 * t + a];
        if (lo) lo[a] = m->tlo[3 * t + a];
        if (hi) hi[a] = m->thi[3 * t + a];
    }
}
