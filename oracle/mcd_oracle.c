/*
 * Plain FP64 CPU oracle for narrow-phase contact detection between rigid
 * particles represented by triangulated meshes (Noble & Weinzierl, "Parallel
 * local time stepping for rigid bodies represented by triangulated meshes").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library calls this code; it exists
 * so that tests and the benchmark's CPU baseline can check the GPU path. It is
 * deliberately slow and direct: world-frame coordinates, double precision
 * everywhere, no blocking, no culling beyond what the definitions state, and
 * it shares no code, header or table with the GPU path. Build with
 * -O2 -ffp-contract=off (no FMA contraction, no fast-math).
 *
 * What it computes, and where the paper defines it:
 *  - Particle motion between snapshots: linear in position, spherical-linear
 *    in the rotation quaternion (section 2, "Physical model"). With a constant
 *    world-frame angular velocity w this is q(t) = exp(t w/2) * q0.
 *  - Contact (section 5, "Geometric model", contact-point definition): two
 *    triangles from different particles are in contact when some point lies
 *    within the halo of both; with halos eps_a, eps_b this holds exactly when
 *    the triangle-triangle distance d <= delta = eps_a + eps_b. The contact
 *    point is the midpoint of the closest points (section 2, "Collision and
 *    update": the point right between the two particles) and the normal is
 *    the shortest distance vector.
 *  - Triangle-triangle distance: the paper defers to known vertex-triangle
 *    and edge-edge code blocks (section 5, "Collision time detection"). The
 *    oracle takes the textbook exact definition: d = 0 if an edge of either
 *    triangle meets the other closed triangle; otherwise the minimum of the 6
 *    vertex-to-triangle and 9 edge-to-edge distances.
 *  - Collision time stamp (section 5, case distinctions and narrowing; the
 *    "widening" remark): per triangle pair the first time in [0, dt] at which
 *    d <= delta, found by sampling the step at S+1 equidistant times, a
 *    Lipschitz rule that excludes crossings between samples, and bisection to
 *    a tolerance, returning the end of the final bracket that is in contact.
 *    Per particle pair the earliest triangle-pair time wins.
 *
 * Readings where the paper is silent are listed with the functions below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ABI 1

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 ld(const double* p) { return mk(p[0], p[1], p[2]); }
static void st(double* p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 crs(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double len2(v3 a) { return dot(a, a); }
static double clamp01(double s) { return s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s); }

int orc_abi_version(void) { return ORC_ABI; }

/* ------------------------------------------------------------------ */
/* Primitive 1: closest point on a closed triangle to a point.          */
/* Voronoi-region classification (vertex, edge and face regions of the  */
/* triangle), as in Ericson, Real-Time Collision Detection, 5.1.5.       */
/* Returns the squared distance; q receives the closest point.           */
/* ------------------------------------------------------------------ */
static double pt_tri(v3 p, v3 a, v3 b, v3 c, v3* q)
{
    v3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { *q = a; return len2(sub(p, *q)); }          /* vertex a */
    v3 bp = sub(p, b);
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { *q = b; return len2(sub(p, *q)); }           /* vertex b */
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {                                /* edge ab */
        double v = d1 / (d1 - d3);
        *q = add(a, scl(ab, v));
        return len2(sub(p, *q));
    }
    v3 cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { *q = c; return len2(sub(p, *q)); }           /* vertex c */
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {                                /* edge ac */
        double w = d2 / (d2 - d6);
        *q = add(a, scl(ac, w));
        return len2(sub(p, *q));
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {                  /* edge bc */
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        *q = add(b, scl(sub(c, b), w));
        return len2(sub(p, *q));
    }
    double den = 1.0 / (va + vb + vc);                                         /* face */
    double v = vb * den, w = vc * den;
    *q = add(a, add(scl(ab, v), scl(ac, w)));
    return len2(sub(p, *q));
}

/* ------------------------------------------------------------------ */
/* Primitive 2: closest points of two segments p1+s*(q1-p1), p2+t*(q2-p2) */
/* with s, t in [0,1]: the infinite-line solution for s clamped to [0,1],  */
/* then t optimal for that s; if t leaves [0,1] it is clamped and s is     */
/* recomputed (Ericson 5.1.9, after Lumelsky 1985). Reading: a denominator */
/* a*e - b*b <= 1e-14*a*e marks parallel segments, where s = 0 is taken    */
/* first. Segments here are triangle edges, never of zero length.          */
/* ------------------------------------------------------------------ */
static double seg_seg(v3 p1, v3 q1, v3 p2, v3 q2, v3* c1, v3* c2)
{
    v3 d1 = sub(q1, p1), d2 = sub(q2, p2), r = sub(p1, p2);
    double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    double c = dot(d1, r), b = dot(d1, d2);
    double den = a * e - b * b;
    double s = 0.0, t;
    if (den > 1e-14 * a * e) s = clamp01((b * f - c * e) / den);
    t = (b * s + f) / e;
    if (t < 0.0) {
        t = 0.0;
        s = clamp01(-c / a);
    } else if (t > 1.0) {
        t = 1.0;
        s = clamp01((b - c) / a);
    }
    *c1 = add(p1, scl(d1, s));
    *c2 = add(p2, scl(d2, t));
    return len2(sub(*c1, *c2));
}

/* ------------------------------------------------------------------ */
/* Primitive 3: does the closed segment pq meet the closed triangle abc?  */
/* Signed volumes: the endpoints must lie on opposite sides of (or on)    */
/* the triangle's plane, and the line pq must pass through the triangle   */
/* (three triple products of one sign, zero allowed). A segment lying in  */
/* the plane is left to the distance features, which are zero for         */
/* coplanar overlap (a vertex inside the other triangle, or crossing      */
/* edges). Reading: "in the plane" means both endpoints lie within        */
/* 1e-12 * l of it, l the largest of |p-a|, |q-a|, |b-a|, |c-a|; there the */
/* triple products are rounding noise, and leaving the case to the        */
/* features changes d by at most about that height.                       */
/* On a hit x is the point where pq crosses the plane.                    */
/* ------------------------------------------------------------------ */
static int seg_tri(v3 p, v3 q, v3 a, v3 b, v3 c, v3* x)
{
    v3 n = crs(sub(b, a), sub(c, a));
    double op = dot(n, sub(p, a)), oq = dot(n, sub(q, a));
    double l = sqrt(len2(sub(p, a)));
    double l2 = sqrt(len2(sub(q, a))), l3 = sqrt(len2(sub(b, a))), l4 = sqrt(len2(sub(c, a)));
    if (l2 > l) l = l2;
    if (l3 > l) l = l3;
    if (l4 > l) l = l4;
    double hmax = 1e-12 * l * sqrt(len2(n));
    if (fabs(op) <= hmax && fabs(oq) <= hmax) return 0;   /* in the plane */
    if ((op > 0.0 && oq > 0.0) || (op < 0.0 && oq < 0.0)) return 0;
    v3 d = sub(q, p);
    double s1 = dot(d, crs(sub(a, p), sub(b, p)));
    double s2 = dot(d, crs(sub(b, p), sub(c, p)));
    double s3 = dot(d, crs(sub(c, p), sub(a, p)));
    int pos = (s1 >= 0.0) && (s2 >= 0.0) && (s3 >= 0.0);
    int neg = (s1 <= 0.0) && (s2 <= 0.0) && (s3 <= 0.0);
    if (!pos && !neg) return 0;
    double t = op / (op - oq);
    *x = add(p, scl(d, t));
    return 1;
}

/* ------------------------------------------------------------------ */
/* Triangle-triangle distance with closest points.                      */
/* Order (fixed; the first strictly smaller value wins):                */
/*   intersections: edges A.e0, A.e1, A.e2 against B, then B's edges    */
/*   against A (e_k joins vertex k and vertex k+1 mod 3) -> d = 0;      */
/*   otherwise vertices A.v0..v2 against B, B.v0..v2 against A, and the */
/*   9 edge pairs (A.e_k, B.e_l) with k the slow index.                 */
/* feature: 0..5 intersection edge, 6..11 vertex, 12..20 edge pair.     */
/* Returns d (not squared).                                             */
/* ------------------------------------------------------------------ */
double orc_tri_tri(const double* A, const double* B, double* pa, double* pb, int* feature)
{
    v3 a[3] = {ld(A), ld(A + 3), ld(A + 6)};
    v3 b[3] = {ld(B), ld(B + 3), ld(B + 6)};
    v3 x, q, c1, c2;
    for (int k = 0; k < 3; ++k)
        if (seg_tri(a[k], a[(k + 1) % 3], b[0], b[1], b[2], &x)) {
            st(pa, x); st(pb, x); if (feature) *feature = k; return 0.0;
        }
    for (int k = 0; k < 3; ++k)
        if (seg_tri(b[k], b[(k + 1) % 3], a[0], a[1], a[2], &x)) {
            st(pa, x); st(pb, x); if (feature) *feature = 3 + k; return 0.0;
        }
    double best = INFINITY;
    v3 ba = a[0], bb = b[0];
    int bf = -1;
    for (int k = 0; k < 3; ++k) {
        double d2 = pt_tri(a[k], b[0], b[1], b[2], &q);
        if (d2 < best) { best = d2; ba = a[k]; bb = q; bf = 6 + k; }
    }
    for (int k = 0; k < 3; ++k) {
        double d2 = pt_tri(b[k], a[0], a[1], a[2], &q);
        if (d2 < best) { best = d2; ba = q; bb = b[k]; bf = 9 + k; }
    }
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double d2 = seg_seg(a[k], a[(k + 1) % 3], b[l], b[(l + 1) % 3], &c1, &c2);
            if (d2 < best) { best = d2; ba = c1; bb = c2; bf = 12 + 3 * k + l; }
        }
    st(pa, ba); st(pb, bb);
    if (feature) *feature = bf;
    return sqrt(best);
}

/* Exposed primitives (for the tests that pin them). */
double orc_point_triangle(const double* p, const double* T, double* q)
{
    v3 r;
    double d2 = pt_tri(ld(p), ld(T), ld(T + 3), ld(T + 6), &r);
    st(q, r);
    return sqrt(d2);
}

double orc_segment_segment(const double* p1, const double* q1, const double* p2,
                           const double* q2, double* c1, double* c2)
{
    v3 a, b;
    double d2 = seg_seg(ld(p1), ld(q1), ld(p2), ld(q2), &a, &b);
    st(c1, a); st(c2, b);
    return sqrt(d2);
}

int orc_segment_triangle(const double* p, const double* q, const double* T, double* x)
{
    v3 r = mk(0, 0, 0);
    int hit = seg_tri(ld(p), ld(q), ld(T), ld(T + 3), ld(T + 6), &r);
    st(x, r);
    return hit;
}

/* ------------------------------------------------------------------ */
/* Rigid motion (section 2, "Physical model"): x(t) = x0 + v t and        */
/* q(t) = exp(t w / 2) * q0 for a constant world-frame angular velocity w, */
/* the constant-rate slerp between two snapshots. R(q) for unit q.         */
/* state: x[3], q[4] = (w, x, y, z), v[3], w[3].                           */
/* ------------------------------------------------------------------ */
void orc_pose(const double* s, double t, double* R, double* xt)
{
    double qw = s[3], qx = s[4], qy = s[5], qz = s[6];
    double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= nq; qx /= nq; qy /= nq; qz /= nq;
    double wx = s[10], wy = s[11], wz = s[12];
    double wn = sqrt(wx * wx + wy * wy + wz * wz);
    if (wn > 0.0 && t != 0.0) {
        double h = 0.5 * wn * t;
        double cw = cos(h), sw = sin(h) / wn;
        double ew = cw, ex = sw * wx, ey = sw * wy, ez = sw * wz;  /* exp(t w/2) */
        double rw = ew * qw - ex * qx - ey * qy - ez * qz;         /* e * q0 */
        double rx = ew * qx + ex * qw + ey * qz - ez * qy;
        double ry = ew * qy - ex * qz + ey * qw + ez * qx;
        double rz = ew * qz + ex * qy - ey * qx + ez * qw;
        qw = rw; qx = rx; qy = ry; qz = rz;
    }
    R[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    R[1] = 2.0 * (qx * qy - qw * qz);
    R[2] = 2.0 * (qx * qz + qw * qy);
    R[3] = 2.0 * (qx * qy + qw * qz);
    R[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    R[5] = 2.0 * (qy * qz - qw * qx);
    R[6] = 2.0 * (qx * qz - qw * qy);
    R[7] = 2.0 * (qy * qz + qw * qx);
    R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
    xt[0] = s[0] + s[7] * t;
    xt[1] = s[1] + s[8] * t;
    xt[2] = s[2] + s[9] * t;
}

/* World-frame triangles (nt x 9) of a mesh at time t. */
static void world_tris(const double* V, const int32_t* F, int nt, const double* s,
                       double t, double* out)
{
    double R[9], x[3];
    orc_pose(s, t, R, x);
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k) {
            const double* p = V + 3 * F[3 * i + k];
            double* o = out + 9 * i + 3 * k;
            for (int r = 0; r < 3; ++r)
                o[r] = x[r] + (R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2]);
        }
}

void orc_world_tris(const double* V, const int32_t* F, int nt, const double* s, double t,
                    double* out)
{
    world_tris(V, F, nt, s, t, out);
}

/* ------------------------------------------------------------------ */
/* Mesh/particle store passed from Python (flat arrays).                */
/* ------------------------------------------------------------------ */
typedef struct {
    const double* V;        /* all vertices, body frame */
    const int32_t* F;       /* all faces, indices local to their mesh */
    const int64_t* voff;    /* per mesh: first vertex */
    const int64_t* toff;    /* per mesh: first face */
    const int32_t* tcount;  /* per mesh: number of faces */
    const double* halo;     /* per mesh */
    const double* radius;   /* per mesh: largest vertex distance from the centre */
    const int32_t* mesh_of; /* per particle */
    const double* state;    /* per particle, 13 doubles */
} orc_store;

/* Contact record (pair index, triangle ids, d, closest points). */
typedef struct {
    int32_t pair, tri_a, tri_b, pad;
    double d, pa[3], pb[3];
} orc_contact;

typedef struct { orc_contact* c; int64_t n, cap; } cbuf;

static void cpush(cbuf* b, const orc_contact* c)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 64;
        b->c = (orc_contact*)realloc(b->c, (size_t)b->cap * sizeof(orc_contact));
    }
    b->c[b->n++] = *c;
}

/* Pair result. status: 0 none, 1 contact at start (AT_START), 2 collides. */
typedef struct {
    double d, pa[3], pb[3], toi;
    int32_t tri_a, tri_b, contact, status;
} orc_pair;

/* ------------------------------------------------------------------ */
/* Static pair query at time t: every triangle pair (i, j), i in A, j in  */
/* B, in row-major order. d_min with the lowest (i, j) on ties; contact   */
/* flag d_min <= delta (closed, "at most" in the contact definition);     */
/* contact set = all (i, j) with d_ij <= delta.                           */
/* ------------------------------------------------------------------ */
static void static_pair(const orc_store* S, int32_t pidx, int32_t pa_id, int32_t pb_id,
                        double t, double* WA, double* WB, orc_pair* out, cbuf* cb)
{
    int ma = S->mesh_of[pa_id], mb = S->mesh_of[pb_id];
    int na = S->tcount[ma], nb = S->tcount[mb];
    double delta = S->halo[ma] + S->halo[mb];
    world_tris(S->V + 3 * S->voff[ma], S->F + 3 * S->toff[ma], na, S->state + 13 * pa_id, t, WA);
    world_tris(S->V + 3 * S->voff[mb], S->F + 3 * S->toff[mb], nb, S->state + 13 * pb_id, t, WB);
    double best = INFINITY;
    double xa[3], xb[3];
    out->tri_a = -1; out->tri_b = -1;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            double d = orc_tri_tri(WA + 9 * i, WB + 9 * j, xa, xb, NULL);
            if (d < best) {
                best = d;
                out->tri_a = i; out->tri_b = j;
                memcpy(out->pa, xa, sizeof xa); memcpy(out->pb, xb, sizeof xb);
            }
            if (d <= delta && cb) {
                orc_contact c;
                c.pair = pidx; c.tri_a = i; c.tri_b = j; c.pad = 0; c.d = d;
                memcpy(c.pa, xa, sizeof xa); memcpy(c.pb, xb, sizeof xb);
                cpush(cb, &c);
            }
        }
    out->d = best;
    out->contact = best <= delta;
}

static int max_tris(const orc_store* S, const int32_t* pairs, int n)
{
    int m = 0;
    for (int p = 0; p < 2 * n; ++p) {
        int k = S->tcount[S->mesh_of[pairs[p]]];
        if (k > m) m = k;
    }
    return m;
}

static int64_t gather(cbuf* bufs, int n, orc_contact* out, int64_t cap)
{
    int64_t tot = 0;
    for (int p = 0; p < n; ++p) {
        for (int64_t k = 0; k < bufs[p].n; ++k) {
            if (tot < cap) out[tot] = bufs[p].c[k];
            ++tot;
        }
        free(bufs[p].c);
    }
    free(bufs);
    return tot;
}

/* Returns the number of contacts (records beyond cap are counted, not written). */
int64_t orc_static_pairs(const double* V, const int32_t* F, const int64_t* voff,
                         const int64_t* toff, const int32_t* tcount, const double* halo,
                         const int32_t* mesh_of, const double* state, int32_t n_pairs,
                         const int32_t* pairs, double t, orc_pair* out,
                         orc_contact* contacts, int64_t cap)
{
    orc_store S = {V, F, voff, toff, tcount, halo, NULL, mesh_of, state};
    int mt = max_tris(&S, pairs, n_pairs);
    cbuf* bufs = (cbuf*)calloc((size_t)(n_pairs > 0 ? n_pairs : 1), sizeof(cbuf));
#pragma omp parallel
    {
        double* WA = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
        double* WB = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < n_pairs; ++p)
            static_pair(&S, p, pairs[2 * p], pairs[2 * p + 1], t, WA, WB, out + p, bufs + p);
        free(WA); free(WB);
    }
    return gather(bufs, n_pairs, contacts, cap);
}

/* ------------------------------------------------------------------ */
/* Collision time stamp (section 5: case distinctions, narrowing and     */
/* widening; motion as above). Readings where the paper is silent:       */
/*  - samples t_k = k*dt/S, k = 0..S (S given, shared with the GPU path); */
/*  - L = |v_a - v_b| + |w_a| R_a + |w_b| R_b bounds how fast any distance */
/*    between the two bodies can change, so on [lo, hi] with end values   */
/*    d_lo, d_hi > delta a crossing is impossible when                   */
/*    (d_lo + d_hi - L (hi - lo)) / 2 > delta;                            */
/*  - an interval that cannot be excluded is halved depth first, left     */
/*    half first, down to width tol; a leaf of width <= tol with both ends */
/*    above delta is a graze and yields no contact;                       */
/*  - an interval whose right end is in contact is bisected (midpoint     */
/*    (lo+hi)/2) until hi - lo <= tol and hi is returned: the first time  */
/*    known to be in contact ("widening" towards a non-zero overlap);     */
/*  - d(0) <= delta gives t = 0 (contact at the start: case 2, which does */
/*    not constrain the step); d(0) - delta > L dt gives no collision.    */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *A, *B;     /* body-frame triangle (9) */
    const double *sa, *sb;   /* states */
    double delta, L, tol;
    int64_t evals, grazes;
} toi_ctx;

static double dist_at(toi_ctx* c, double t)
{
    double Ra[9], xa[3], Rb[9], xb[3], WA[9], WB[9], p[3], q[3];
    orc_pose(c->sa, t, Ra, xa);
    orc_pose(c->sb, t, Rb, xb);
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r) {
            const double* u = c->A + 3 * k;
            const double* w = c->B + 3 * k;
            WA[3 * k + r] = xa[r] + (Ra[3 * r] * u[0] + Ra[3 * r + 1] * u[1] + Ra[3 * r + 2] * u[2]);
            WB[3 * k + r] = xb[r] + (Rb[3 * r] * w[0] + Rb[3 * r + 1] * w[1] + Rb[3 * r + 2] * w[2]);
        }
    c->evals++;
    return orc_tri_tri(WA, WB, p, q, NULL);
}

static double bisect(toi_ctx* c, double lo, double hi)
{
    while (hi - lo > c->tol) {
        double mid = (lo + hi) * 0.5;
        if (dist_at(c, mid) <= c->delta) hi = mid; else lo = mid;
    }
    return hi;
}

/* First contact time in [lo, hi] given d(lo) = dlo > delta and d(hi) = dhi. */
static double interval(toi_ctx* c, double lo, double hi, double dlo, double dhi)
{
    if (dhi <= c->delta) return bisect(c, lo, hi);
    if ((dlo + dhi - c->L * (hi - lo)) * 0.5 > c->delta) return INFINITY;
    if (hi - lo <= c->tol) { c->grazes++; return INFINITY; }
    double mid = (lo + hi) * 0.5;
    double dm = dist_at(c, mid);
    double r = interval(c, lo, mid, dlo, dm);
    if (r < INFINITY) return r;
    return interval(c, mid, hi, dm, dhi);
}

double orc_tri_pair_toi(const double* A, const double* B, const double* sa, const double* sb,
                        double delta, double L, double dt, int32_t S, double tol,
                        int64_t* evals, int64_t* grazes)
{
    toi_ctx c = {A, B, sa, sb, delta, L, tol, 0, 0};
    double r = INFINITY;
    double d0 = dist_at(&c, 0.0);
    if (d0 <= delta) r = 0.0;
    else if (d0 - delta > L * dt) r = INFINITY;
    else {
        double dprev = d0;
        for (int k = 0; k < S; ++k) {
            double t0 = (double)k * dt / (double)S;
            double t1 = (double)(k + 1) * dt / (double)S;
            double d1 = dist_at(&c, t1);
            r = interval(&c, t0, t1, dprev, d1);
            if (r < INFINITY) break;
            dprev = d1;
        }
    }
    if (evals) *evals += c.evals;
    if (grazes) *grazes += c.grazes;
    return r;
}

static void tri_body(const orc_store* S, int m, int i, double* out)
{
    const double* V = S->V + 3 * S->voff[m];
    const int32_t* F = S->F + 3 * (S->toff[m] + i);
    for (int k = 0; k < 3; ++k) memcpy(out + 3 * k, V + 3 * F[k], 3 * sizeof(double));
}

static void toi_pair(const orc_store* S, int32_t pidx, int32_t ia, int32_t ib, double dt,
                     int32_t nS, double tol_rel, double* WA, double* WB, orc_pair* out,
                     cbuf* cb, int64_t* evals, int64_t* grazes)
{
    int ma = S->mesh_of[ia], mb = S->mesh_of[ib];
    int na = S->tcount[ma], nb = S->tcount[mb];
    const double *sa = S->state + 13 * ia, *sb = S->state + 13 * ib;
    double delta = S->halo[ma] + S->halo[mb];
    v3 dv = sub(ld(sa + 7), ld(sb + 7));
    double L = sqrt(len2(dv)) + sqrt(len2(ld(sa + 10))) * S->radius[ma]
             + sqrt(len2(ld(sb + 10))) * S->radius[mb];
    double tol = tol_rel * dt;
    double best = INFINITY;
    int bi = -1, bj = -1;
    double A[9], B[9];
    for (int i = 0; i < na; ++i) {
        tri_body(S, ma, i, A);
        for (int j = 0; j < nb; ++j) {
            tri_body(S, mb, j, B);
            double tij = orc_tri_pair_toi(A, B, sa, sb, delta, L, dt, nS, tol, evals, grazes);
            if (tij < best) { best = tij; bi = i; bj = j; }
        }
    }
    out->toi = best;
    if (best == INFINITY) {
        out->status = 0; out->contact = 0;
        out->tri_a = -1; out->tri_b = -1; out->d = INFINITY;
        memset(out->pa, 0, sizeof out->pa); memset(out->pb, 0, sizeof out->pb);
        return;
    }
    out->status = best == 0.0 ? 1 : 2;
    /* Contact records at the pair's time stamp (static query at t*). */
    orc_pair tmp;
    static_pair(S, pidx, ia, ib, best, WA, WB, &tmp, cb);
    out->contact = 1;
    out->tri_a = bi; out->tri_b = bj;
    /* Distance and closest points of the winning triangle pair at t*. */
    out->d = orc_tri_tri(WA + 9 * bi, WB + 9 * bj, out->pa, out->pb, NULL);
}

int64_t orc_toi_pairs(const double* V, const int32_t* F, const int64_t* voff,
                      const int64_t* toff, const int32_t* tcount, const double* halo,
                      const double* radius, const int32_t* mesh_of, const double* state,
                      int32_t n_pairs, const int32_t* pairs, double dt, int32_t nS,
                      double tol_rel, orc_pair* out, orc_contact* contacts, int64_t cap,
                      int64_t* diag /* [evals, grazes] */)
{
    orc_store S = {V, F, voff, toff, tcount, halo, radius, mesh_of, state};
    int mt = max_tris(&S, pairs, n_pairs);
    cbuf* bufs = (cbuf*)calloc((size_t)(n_pairs > 0 ? n_pairs : 1), sizeof(cbuf));
    int64_t ev = 0, gr = 0;
#pragma omp parallel reduction(+ : ev, gr)
    {
        double* WA = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
        double* WB = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < n_pairs; ++p)
            toi_pair(&S, p, pairs[2 * p], pairs[2 * p + 1], dt, nS, tol_rel, WA, WB, out + p,
                     bufs + p, &ev, &gr);
        free(WA); free(WB);
    }
    if (diag) { diag[0] = ev; diag[1] = gr; }
    return gather(bufs, n_pairs, contacts, cap);
}

/* ------------------------------------------------------------------ */
/* Broad phase and clusters of a particle set (section 3).                */
/* Each particle is its bounding sphere about the rotation centre, radius */
/* r = R + eps (largest vertex distance plus halo), moving linearly from  */
/* x at the start to x + v dt at the end of the step.                     */
/* Check 1 (space-time bounding boxes): the box around both snapshots of  */
/* each sphere; boxes that do not overlap rule the pair out.              */
/* Check 2 (space-time tubes): the two spheres at a common time t in      */
/* [0, dt]; the pair stays when their centres come within r_a + r_b at    */
/* the time of closest approach of the two linear paths (clamped to the   */
/* step).                                                                 */
/* Clusters (the unconnected subgraphs): every particle starts with its   */
/* own position as label and takes the smallest label among itself and   */
/* its partners, sweep after sweep, until a sweep changes nothing. Reading */
/* of the paper's colouring rule: its "plus one" would never settle into  */
/* one label per subgraph, so the label is the plain minimum.             */
/* x, v: n*3 (centre, velocity); r: n radii. pairs_out: 2*cap positions  */
/* (a < b), ordered by a then b. label: n (the smallest position of the   */
/* particle's subgraph). Returns the pair count (pairs beyond cap are     */
/* counted, not written); sweeps receives the sweeps run.                 */
/* ------------------------------------------------------------------ */
static int box_overlap(const double* xa, const double* va, double ra, const double* xb,
                       const double* vb, double rb, double dt)
{
    for (int c = 0; c < 3; ++c) {
        double a0 = xa[c], a1 = xa[c] + va[c] * dt, b0 = xb[c], b1 = xb[c] + vb[c] * dt;
        double alo = (a0 < a1 ? a0 : a1) - ra, ahi = (a0 > a1 ? a0 : a1) + ra;
        double blo = (b0 < b1 ? b0 : b1) - rb, bhi = (b0 > b1 ? b0 : b1) + rb;
        if (alo > bhi || blo > ahi) return 0;
    }
    return 1;
}

static int tubes_meet(const double* xa, const double* va, double ra, const double* xb,
                      const double* vb, double rb, double dt)
{
    double d[3], w[3], ww = 0.0, dw = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = xb[c] - xa[c];
        w[c] = vb[c] - va[c];
        ww += w[c] * w[c];
        dw += d[c] * w[c];
    }
    double t = 0.0;
    if (dt > 0.0 && ww > 0.0) {
        t = -dw / ww;
        if (t < 0.0) t = 0.0;
        if (t > dt) t = dt;
    }
    double e2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double e = d[c] + w[c] * t;
        e2 += e * e;
    }
    return e2 <= (ra + rb) * (ra + rb);
}

int64_t orc_broad_phase(int32_t n, const double* x, const double* v, const double* r, double dt,
                        int32_t* pairs_out, int64_t cap, int32_t* label, int32_t* sweeps)
{
    int64_t np = 0;
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            if (!box_overlap(x + 3 * a, v + 3 * a, r[a], x + 3 * b, v + 3 * b, r[b], dt)) continue;
            if (!tubes_meet(x + 3 * a, v + 3 * a, r[a], x + 3 * b, v + 3 * b, r[b], dt)) continue;
            if (np < cap) { pairs_out[2 * np] = a; pairs_out[2 * np + 1] = b; }
            ++np;
        }
    if (label) {
        const int64_t m = np < cap ? np : cap;
        int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int i = 0; i < n; ++i) label[i] = i;
        int k = 0, changed = 1;
        while (changed) {
            changed = 0;
            ++k;
            for (int i = 0; i < n; ++i) next[i] = label[i];
            for (int64_t e = 0; e < m; ++e) {
                int a = pairs_out[2 * e], b = pairs_out[2 * e + 1];
                if (label[b] < next[a]) next[a] = label[b];
                if (label[a] < next[b]) next[b] = label[a];
            }
            for (int i = 0; i < n; ++i) {
                if (next[i] != label[i]) changed = 1;
                label[i] = next[i];
            }
        }
        if (sweeps) *sweeps = k;
        free(next);
    }
    return np;
}

/* ------------------------------------------------------------------ */
/* Narrowing (section 5, "Collision time detection": the iterative        */
/* narrowing of the time span with the analytic vertex-triangle test and  */
/* sampled edge-edge distances). Rotation is neglected, as the paper says */
/* of this approximation: each triangle keeps its orientation at the start */
/* and moves with its particle's velocity. With the span [0, T]:           */
/*  - vertex-triangle (3 vertices of each triangle against the other       */
/*    triangle): in the frame moving with the triangle the vertex moves on */
/*    a line from its start to its end position; the distance to the       */
/*    triangle is evaluated at the start, at the end and, when the line    */
/*    crosses the triangle's plane inside the span, at the crossing;       */
/*  - edge-edge (9 pairs): the distance at the start, the middle and the   */
/*    end of the span;                                                     */
/*  - a feature is in contact at the earliest of its evaluation times with */
/*    distance <= delta; the triangle pair's time is the earliest over its */
/*    15 features, and the particle pair's the earliest over all triangle  */
/*    pairs (lowest (i, j) on ties);                                       */
/*  - while that time is earlier than T, T becomes that time and the tests */
/*    run again; the final T is the pair's time stamp.                     */
/* Readings: the "distance in-between" of an edge pair is its distance at */
/* the middle of the span; the narrowing runs per particle pair (a        */
/* cluster's time is the earliest of its pairs'); no widening is applied; */
/* at most 200 rounds. Status: none when the first round finds no contact, */
/* at the start when the time is 0, else collides. Contacts are reported  */
/* at the final time with the same translation-only motion.               */
/* ------------------------------------------------------------------ */
typedef struct { v3 p[3]; } tri3;

static tri3 ld_tri(const double* T)
{
    tri3 r;
    for (int k = 0; k < 3; ++k) r.p[k] = ld(T + 3 * k);
    return r;
}

/* Earliest s in {0, s_plane, 1} (s_plane only inside (0, 1)) at which the
 * point p + s w is within delta of triangle t; returns 2 when none is. */
static double vert_tri_time(v3 p, v3 w, tri3 t, double delta)
{
    v3 q;
    v3 n = crs(sub(t.p[1], t.p[0]), sub(t.p[2], t.p[0]));
    double cand[3];
    int nc = 0;
    cand[nc++] = 0.0;
    double wn = dot(w, n);
    if (wn != 0.0) {
        double s = -dot(sub(p, t.p[0]), n) / wn;
        if (s > 0.0 && s < 1.0) cand[nc++] = s;
    }
    cand[nc++] = 1.0;
    for (int k = 0; k < nc; ++k)
        if (pt_tri(add(p, scl(w, cand[k])), t.p[0], t.p[1], t.p[2], &q) <= delta * delta) return cand[k];
    return 2.0;
}

/* Earliest s in {0, 1/2, 1} at which segment (a0, a1) and segment (b0, b1)
 * moved by s w are within delta; 2 when none is. */
static double edge_edge_time(v3 a0, v3 a1, v3 b0, v3 b1, v3 w, double delta)
{
    static const double ss[3] = {0.0, 0.5, 1.0};
    v3 c1, c2;
    for (int k = 0; k < 3; ++k) {
        v3 d = scl(w, ss[k]);
        if (seg_seg(a0, a1, add(b0, d), add(b1, d), &c1, &c2) <= delta * delta) return ss[k];
    }
    return 2.0;
}

/* One round for a triangle pair: the earliest contact as a fraction of the
 * span (2: none). A, B: triangles at the start; w: B's displacement relative
 * to A over the span. */
double orc_narrow_tri_pair(const double* A, const double* B, const double* w_rel, double delta)
{
    tri3 a = ld_tri(A), b = ld_tri(B);
    v3 w = ld(w_rel), mw = scl(w, -1.0);
    double best = 2.0;
    for (int k = 0; k < 3; ++k) {
        double s = vert_tri_time(a.p[k], mw, b, delta);   /* A's vertex, frame of B */
        if (s < best) best = s;
    }
    for (int k = 0; k < 3; ++k) {
        double s = vert_tri_time(b.p[k], w, a, delta);    /* B's vertex, frame of A */
        if (s < best) best = s;
    }
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double s = edge_edge_time(a.p[k], a.p[(k + 1) % 3], b.p[l], b.p[(l + 1) % 3], w, delta);
            if (s < best) best = s;
        }
    return best;
}

static void narrow_pair(const orc_store* S, int32_t pidx, int32_t ia, int32_t ib, double dt,
                        double* WA, double* WB, orc_pair* out, cbuf* cb, int32_t* rounds)
{
    int ma = S->mesh_of[ia], mb = S->mesh_of[ib];
    int na = S->tcount[ma], nb = S->tcount[mb];
    const double *sa = S->state + 13 * ia, *sb = S->state + 13 * ib;
    double delta = S->halo[ma] + S->halo[mb];
    world_tris(S->V + 3 * S->voff[ma], S->F + 3 * S->toff[ma], na, sa, 0.0, WA);
    world_tris(S->V + 3 * S->voff[mb], S->F + 3 * S->toff[mb], nb, sb, 0.0, WB);
    v3 vrel = sub(ld(sb + 7), ld(sa + 7));
    double T = dt;
    int found = 0, r = 0;
    int bi = -1, bj = -1;
    for (r = 1; r <= 200; ++r) {
        v3 w = scl(vrel, T);
        double wa[3];
        st(wa, w);
        double tmin = INFINITY;
        int ti = -1, tj = -1;
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j) {
                double s = orc_narrow_tri_pair(WA + 9 * i, WB + 9 * j, wa, delta);
                if (s > 1.0) continue;
                double t = s * T;
                if (t < tmin) { tmin = t; ti = i; tj = j; }
            }
        if (tmin == INFINITY) break;          /* no contact in this span */
        found = 1;
        bi = ti; bj = tj;
        if (!(tmin < T)) break;               /* nothing earlier: T stays */
        T = tmin;
    }
    if (rounds) *rounds = r;
    if (!found) {
        out->toi = INFINITY; out->status = 0; out->contact = 0;
        out->tri_a = -1; out->tri_b = -1; out->d = INFINITY;
        memset(out->pa, 0, sizeof out->pa); memset(out->pb, 0, sizeof out->pb);
        return;
    }
    out->toi = T;
    out->status = T == 0.0 ? 1 : 2;
    out->contact = 1;
    out->tri_a = bi; out->tri_b = bj;
    /* translation-only poses at T: the states without angular velocity */
    double ta[13], tb[13];
    memcpy(ta, sa, sizeof ta); memcpy(tb, sb, sizeof tb);
    ta[10] = ta[11] = ta[12] = 0.0;
    tb[10] = tb[11] = tb[12] = 0.0;
    orc_store S2 = *S;
    double* st2 = (double*)malloc(sizeof(double) * 13 * 2);
    memcpy(st2, ta, sizeof ta); memcpy(st2 + 13, tb, sizeof tb);
    int32_t mo[2] = {ma, mb};
    S2.state = st2;
    S2.mesh_of = mo;
    orc_pair tmp;
    static_pair(&S2, pidx, 0, 1, T, WA, WB, &tmp, cb);
    out->d = orc_tri_tri(WA + 9 * bi, WB + 9 * bj, out->pa, out->pb, NULL);
    free(st2);
}

int64_t orc_narrow_pairs(const double* V, const int32_t* F, const int64_t* voff,
                         const int64_t* toff, const int32_t* tcount, const double* halo,
                         const int32_t* mesh_of, const double* state, int32_t n_pairs,
                         const int32_t* pairs, double dt, orc_pair* out, orc_contact* contacts,
                         int64_t cap, int32_t* rounds)
{
    orc_store S = {V, F, voff, toff, tcount, halo, NULL, mesh_of, state};
    int mt = max_tris(&S, pairs, n_pairs);
    cbuf* bufs = (cbuf*)calloc((size_t)(n_pairs > 0 ? n_pairs : 1), sizeof(cbuf));
#pragma omp parallel
    {
        double* WA = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
        double* WB = (double*)malloc((size_t)mt * 9 * sizeof(double) + 8);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < n_pairs; ++p)
            narrow_pair(&S, p, pairs[2 * p], pairs[2 * p + 1], dt, WA, WB, out + p, bufs + p,
                        rounds ? rounds + p : NULL);
        free(WA); free(WB);
    }
    return gather(bufs, n_pairs, contacts, cap);
}

/* ------------------------------------------------------------------ */
/* Contact fusion (section 5, after the contact-point definition: contact */
/* points close in space are fused into one, which also centres them      */
/* within parallel triangles). Reading: per particle pair, over its       */
/* records in (tri_a, tri_b) order, the first record not yet in a group   */
/* seeds one and every later free record whose contact point (midpoint of */
/* its closest points) lies within the pair's threshold delta[pair] of    */
/* the seed's joins it. A group becomes one record: the seed's pair and   */
/* triangles; contact point = mean of the members' contact points (summed */
/* in record order); distance vector and d of the member with the smallest */
/* d (first on ties), placed about that mean; pad = number of members.    */
/* in: n records sorted by (pair, tri_a, tri_b); out: at most n records.  */
/* Returns the number of fused records.                                   */
/* ------------------------------------------------------------------ */
int64_t orc_fuse_contacts(const orc_contact* in, int64_t n, const double* delta, orc_contact* out)
{
    int64_t nout = 0;
    char* used = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t lo = 0;
    while (lo < n) {
        int64_t hi = lo;
        while (hi < n && in[hi].pair == in[lo].pair) ++hi;
        double r2 = delta[in[lo].pair] * delta[in[lo].pair];
        for (int64_t s = lo; s < hi; ++s) {
            if (used[s]) continue;
            v3 xs = scl(add(ld(in[s].pa), ld(in[s].pb)), 0.5);
            v3 sum = mk(0, 0, 0);
            int cnt = 0;
            int64_t best = s;
            for (int64_t k = s; k < hi; ++k) {
                if (used[k]) continue;
                v3 x = scl(add(ld(in[k].pa), ld(in[k].pb)), 0.5);
                if (k != s && len2(sub(x, xs)) > r2) continue;
                used[k] = 1;
                sum = add(sum, x);
                ++cnt;
                if (in[k].d < in[best].d) best = k;
            }
            orc_contact f = in[s];
            v3 mean = scl(sum, 1.0 / cnt);
            v3 h = scl(sub(ld(in[best].pb), ld(in[best].pa)), 0.5);
            st(f.pa, sub(mean, h));
            st(f.pb, add(mean, h));
            f.d = in[best].d;
            f.pad = cnt;
            out[nout++] = f;
        }
        lo = hi;
    }
    free(used);
    return nout;
}

/* ------------------------------------------------------------------ */
/* Particle interaction (section 6): the impulses exchanged at the     */
/* contact points of a cluster, by a Picard iteration that updates the */
/* contribution of one contact point at a time.                        */
/*                                                                    */
/* Mass properties: a closed, consistently oriented triangle mesh of   */
/* unit density; mass, centre of mass and inertia tensor about it from */
/* the divergence theorem, summed over the tetrahedra between the      */
/* origin and each face (tetrahedron 0, a, b, c: volume a.(b x c)/6,   */
/* first moment volume (a+b+c)/4, second moment                         */
/* volume/20 (aa' + bb' + cc' + ss'), s = a+b+c). Inward-facing meshes  */
/* give a negative volume and are taken by absolute value.             */
/*                                                                    */
/* Readings where section 6 is silent:                                  */
/*  - the contact point is the midpoint of the closest points and the  */
/*    normal n points from particle a to b along pb - pa; when pb = pa  */
/*    (intersecting triangles) it points from a's centre of mass to b's; */
/*  - the constraint is on the separation speed of the contact points,  */
/*    u_n = (u_b - u_a).n >= target, target = max(0, -e u_n0) with      */
/*    u_n0 the speed before the solve and e the restitution (e = 0 is   */
/*    the constraint as the paper states it); the normal impulse is     */
/*    non-negative (the penalty that enforces the constraint weakly is  */
/*    replaced by this projection);                                      */
/*  - Coulomb friction: a tangential impulse opposing the sliding       */
/*    velocity, its length at most mu times the normal impulse;        */
/*  - damping: each update moves an impulse by a fraction relax of the  */
/*    way to its new value;                                             */
/*  - the iteration ends after the first sweep whose largest change of  */
/*    a contact's impulse (normal plus tangential length) is at most    */
/*    tol times the largest impulse, or after max_iter sweeps;          */
/*  - order (the paper's colouring): contacts are coloured greedily in  */
/*    their order, each taking the smallest colour that no earlier      */
/*    contact sharing a particle has; a sweep runs the colours in turn  */
/*    and the contacts of a colour in their order (contacts of one      */
/*    colour share no particle, so any order gives the same result);    */
/*  - clusters (the connected components of the contact graph) are      */
/*    independent: each iterates, and stops, on its own.               */
/* ------------------------------------------------------------------ */
int orc_mass_properties(const double* V, const int32_t* F, int32_t nt, double* mass, double* com,
                        double* inertia)
{
    double m = 0.0, f[3] = {0, 0, 0}, C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t t = 0; t < nt; ++t) {
        v3 a = ld(V + 3 * F[3 * t]), b = ld(V + 3 * F[3 * t + 1]), c = ld(V + 3 * F[3 * t + 2]);
        double vol = dot(a, crs(b, c)) / 6.0;
        v3 s = add(add(a, b), c);
        m += vol;
        f[0] += vol * s.x / 4.0; f[1] += vol * s.y / 4.0; f[2] += vol * s.z / 4.0;
        double P[4][3] = {{a.x, a.y, a.z}, {b.x, b.y, b.z}, {c.x, c.y, c.z}, {s.x, s.y, s.z}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += P[k][i] * P[k][j];
                C[3 * i + j] += vol / 20.0 * acc;
            }
    }
    if (m < 0.0) {
        m = -m;
        for (int i = 0; i < 3; ++i) f[i] = -f[i];
        for (int i = 0; i < 9; ++i) C[i] = -C[i];
    }
    if (!(m > 0.0)) return -1;
    double cx = f[0] / m, cy = f[1] / m, cz = f[2] / m;
    double tr = C[0] + C[4] + C[8];
    double cc[3] = {cx, cy, cz}, c2 = cx * cx + cy * cy + cz * cz;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double io = (i == j ? tr : 0.0) - C[3 * i + j];            /* about the origin */
            inertia[3 * i + j] = io - m * ((i == j ? c2 : 0.0) - cc[i] * cc[j]);   /* about the centre */
        }
    *mass = m;
    com[0] = cx; com[1] = cy; com[2] = cz;
    return 0;
}

typedef struct {
    double restitution, friction, relax, tol;
    int32_t max_iter, pad;
} orc_impulse_opts;

typedef struct {
    double invm;
    double Iinv[9];       /* world-frame inverse inertia about the centre of mass */
    v3 xc, rc, vc, w;     /* centre of mass, its offset from the state's origin, velocities */
} imp_body;

static v3 mat_vec(const double* M, v3 a)
{
    return mk(M[0] * a.x + M[1] * a.y + M[2] * a.z, M[3] * a.x + M[4] * a.y + M[5] * a.z,
              M[6] * a.x + M[7] * a.y + M[8] * a.z);
}

/* Inverse of a symmetric positive definite 3x3 matrix by cofactors. */
static void inv3(const double* A, double* B)
{
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    B[0] = c00 / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = c01 / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = c02 / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

/* Velocity of the material point at X. */
static v3 point_vel(const imp_body* b, v3 X) { return add(b->vc, crs(b->w, sub(X, b->xc))); }

/* Impulse J at X on body b. */
static void push(imp_body* b, v3 X, v3 J)
{
    b->vc = add(b->vc, scl(J, b->invm));
    b->w = add(b->w, mat_vec(b->Iinv, crs(sub(X, b->xc), J)));
}

/* n . ((Iinv (r x n)) x r): the rotational part of the effective inverse mass along n. */
static double ang_term(const imp_body* b, v3 X, v3 n)
{
    v3 r = sub(X, b->xc);
    return dot(n, crs(mat_vec(b->Iinv, crs(r, n)), r));
}

int32_t orc_impulses(int32_t np, const double* mass, const double* com, const double* inertia,
                     const double* state, int32_t nc, const int32_t* ab, const double* pa,
                     const double* pb, const orc_impulse_opts* o, double* impulse, double* vel,
                     int32_t* color)
{
    imp_body* B = (imp_body*)calloc((size_t)(np > 0 ? np : 1), sizeof(imp_body));
    for (int32_t i = 0; i < np; ++i) {
        const double* s = state + 13 * i;
        double R[9], x[3], Ib[9], Ibi[9], T[9];
        orc_pose(s, 0.0, R, x);
        B[i].invm = 1.0 / mass[i];
        B[i].rc = mat_vec(R, ld(com + 3 * i));
        B[i].xc = add(ld(x), B[i].rc);
        B[i].w = ld(s + 10);
        B[i].vc = add(ld(s + 7), crs(B[i].w, B[i].rc));
        memcpy(Ib, inertia + 9 * i, sizeof Ib);
        inv3(Ib, Ibi);
        /* R Ibi R' */
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Ibi[3 * r + k] * R[3 * c + k];
                T[3 * r + c] = acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * r + k] * T[3 * k + c];
                B[i].Iinv[3 * r + c] = acc;
            }
    }
    v3* X = (v3*)malloc(sizeof(v3) * (size_t)(nc > 0 ? nc : 1));
    v3* N = (v3*)malloc(sizeof(v3) * (size_t)(nc > 0 ? nc : 1));
    double* un0 = (double*)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double* ln = (double*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    v3* lt = (v3*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(v3));
    int32_t ncol = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const imp_body *A = B + ab[2 * c], *Bb = B + ab[2 * c + 1];
        v3 p = ld(pa + 3 * c), q = ld(pb + 3 * c);
        X[c] = scl(add(p, q), 0.5);
        v3 dv = sub(q, p);
        double d = sqrt(len2(dv));
        if (d > 0.0) {
            N[c] = scl(dv, 1.0 / d);
        } else {
            v3 e = sub(Bb->xc, A->xc);
            double de = sqrt(len2(e));
            N[c] = de > 0.0 ? scl(e, 1.0 / de) : mk(0.0, 0.0, 1.0);
        }
        un0[c] = dot(sub(point_vel(Bb, X[c]), point_vel(A, X[c])), N[c]);
    }
    /* greedy colours: each contact takes the smallest colour that no earlier
       contact sharing one of its particles has (the colours taken at each
       particle are kept as a bit set, grown as needed) */
    int32_t words = 1;
    uint64_t* taken = (uint64_t*)calloc((size_t)(np > 0 ? np : 1) * words, sizeof(uint64_t));
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t a = ab[2 * c], b = ab[2 * c + 1];
        int32_t k = 0;
        while (k < 64 * words && (((taken[(size_t)a * words + k / 64] | taken[(size_t)b * words + k / 64]) >>
                                   (k % 64)) & 1u))
            ++k;
        if (k >= 64 * words) {   /* grow every particle's set */
            uint64_t* t2 = (uint64_t*)calloc((size_t)(np > 0 ? np : 1) * 2 * words, sizeof(uint64_t));
            for (int32_t i = 0; i < np; ++i) memcpy(t2 + (size_t)i * 2 * words, taken + (size_t)i * words, 8 * (size_t)words);
            free(taken);
            taken = t2;
            words *= 2;
        }
        taken[(size_t)a * words + k / 64] |= 1ull << (k % 64);
        taken[(size_t)b * words + k / 64] |= 1ull << (k % 64);
        color[c] = k;
        if (k + 1 > ncol) ncol = k + 1;
    }
    free(taken);
    /* clusters: connected components of the contact graph (union-find) */
    int32_t* up = (int32_t*)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    for (int32_t i = 0; i < np; ++i) up[i] = i;
    for (int32_t c = 0; c < nc; ++c) {
        int32_t x = ab[2 * c], y = ab[2 * c + 1];
        while (up[x] != x) x = up[x];
        while (up[y] != y) y = up[y];
        if (x != y) up[x > y ? x : y] = x < y ? x : y;
    }
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    for (int32_t c = 0; c < nc; ++c) {
        int32_t x = ab[2 * c];
        while (up[x] != x) x = up[x];
        comp[c] = x;
    }
    /* the contacts of each cluster in the order a sweep visits them: by
       colour, then by index (a counting sort over (cluster root, colour)) */
    int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    int64_t* cnt = (int64_t*)calloc((size_t)(np > 0 ? np : 1) * ncol + 1, sizeof(int64_t));
    for (int32_t c = 0; c < nc; ++c) ++cnt[(size_t)comp[c] * ncol + color[c] + 1];
    for (int64_t i = 0; i < (int64_t)np * ncol; ++i) cnt[i + 1] += cnt[i];
    for (int32_t c = 0; c < nc; ++c) seq[cnt[(size_t)comp[c] * ncol + color[c]]++] = c;
    free(cnt);
    const double e = o->restitution, mu = o->friction, relax = o->relax;
    int32_t most = 0;
    for (int32_t lo = 0; lo < nc;) {
        const int32_t root = comp[seq[lo]];
        int32_t hi = lo;
        while (hi < nc && comp[seq[hi]] == root) ++hi;
        int32_t it = 0;
        while (it < o->max_iter) {
            ++it;
            double maxd = 0.0;
            for (int32_t r = lo; r < hi; ++r) {
                const int32_t c = seq[r];
                imp_body *A = B + ab[2 * c], *Bb = B + ab[2 * c + 1];
                v3 x = X[c], n = N[c];
                double un = dot(sub(point_vel(Bb, x), point_vel(A, x)), n);
                double kn = A->invm + Bb->invm + ang_term(A, x, n) + ang_term(Bb, x, n);
                double target = -e * un0[c];
                if (target < 0.0) target = 0.0;
                double star = ln[c] + (target - un) / kn;
                if (star < 0.0) star = 0.0;
                double nl = ln[c] + relax * (star - ln[c]);
                double dl = nl - ln[c];
                ln[c] = nl;
                push(Bb, x, scl(n, dl));
                push(A, x, scl(n, -dl));
                double change = fabs(dl);
                if (mu > 0.0) {
                    v3 u = sub(point_vel(Bb, x), point_vel(A, x));
                    v3 ut = sub(u, scl(n, dot(u, n)));
                    double s = sqrt(len2(ut));
                    v3 trial = lt[c];
                    if (s > 0.0) {
                        v3 t = scl(ut, 1.0 / s);
                        double kt = A->invm + Bb->invm + ang_term(A, x, t) + ang_term(Bb, x, t);
                        trial = sub(lt[c], scl(ut, 1.0 / kt));
                    }
                    double cap = mu * ln[c], tl = sqrt(len2(trial));
                    if (tl > cap) trial = tl > 0.0 ? scl(trial, cap / tl) : trial;
                    v3 nt = add(lt[c], scl(sub(trial, lt[c]), relax));
                    v3 dt = sub(nt, lt[c]);
                    lt[c] = nt;
                    push(Bb, x, dt);
                    push(A, x, scl(dt, -1.0));
                    change += sqrt(len2(dt));
                }
                if (change > maxd) maxd = change;
            }
            double maxl = 0.0;
            for (int32_t r = lo; r < hi; ++r) {
                double l = ln[seq[r]] + sqrt(len2(lt[seq[r]]));
                if (l > maxl) maxl = l;
            }
            if (maxd <= o->tol * maxl) break;
        }
        if (it > most) most = it;
        lo = hi;
    }
    free(seq);
    free(up);
    free(comp);
    for (int32_t c = 0; c < nc; ++c) {
        impulse[4 * c] = ln[c];
        impulse[4 * c + 1] = lt[c].x; impulse[4 * c + 2] = lt[c].y; impulse[4 * c + 3] = lt[c].z;
    }
    for (int32_t i = 0; i < np; ++i) {
        v3 v = sub(B[i].vc, crs(B[i].w, B[i].rc));
        st(vel + 6 * i, v);
        st(vel + 6 * i + 3, B[i].w);
    }
    free(B); free(X); free(N); free(un0); free(ln); free(lt);
    return most;
}
