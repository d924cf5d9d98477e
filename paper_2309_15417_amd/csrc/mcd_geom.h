// Triangle-pair distance on gfx950, templated on float (filter) and double
// (exact). The distance of two triangles is 0 when an edge of one meets the
// other (closed) triangle, otherwise the smallest of: each vertex to the other
// triangle's face when its projection falls inside the face, and the 9
// edge-edge distances. A vertex whose projection falls outside the face is
// nearer to an edge of that face, which an edge pair containing the vertex
// already measures, so the face test needs no edge or vertex regions.
// The contact-point definition (section 5, "Geometric model") needs d and the
// closest points; the exact variant reproduces the winning feature.
#pragma once

#include <hip/hip_runtime.h>

namespace mcd {

template <typename T> struct R3 { T x, y, z; };

template <typename T> __device__ __forceinline__ R3<T> operator-(R3<T> a, R3<T> b)
{ return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> __device__ __forceinline__ R3<T> operator+(R3<T> a, R3<T> b)
{ return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> __device__ __forceinline__ R3<T> operator*(R3<T> a, T s)
{ return {a.x * s, a.y * s, a.z * s}; }
template <typename T> __device__ __forceinline__ T dot(R3<T> a, R3<T> b)
{ return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T> __device__ __forceinline__ R3<T> cross(R3<T> a, R3<T> b)
{ return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Clamp to [0, 1] in one instruction (median of three in FP32, min and max in
// FP64); equal to the comparison form for every finite s.
template <typename T> __device__ __forceinline__ T clamp01(T s);
template <> __device__ __forceinline__ float clamp01<float>(float s) { return __builtin_amdgcn_fmed3f(s, 0.f, 1.f); }
template <> __device__ __forceinline__ double clamp01<double>(double s) { return fmin(fmax(s, 0.0), 1.0); }

template <typename T> __device__ __forceinline__ T recip(T x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T rsq(T x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

// Square root for FP32 filters: the hardware instruction (1 ulp) instead of
// the correctly rounded sequence; every caller compares the result against a
// threshold widened by the FP32 margin mu, hundreds of ulps.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
template <typename T> __device__ __forceinline__ T root(T x);
template <> __device__ __forceinline__ float root<float>(float x) { return fsqrt(x); }
template <> __device__ __forceinline__ double root<double>(double x) { return sqrt(x); }

template <typename T> __device__ __forceinline__ T big();
template <> __device__ __forceinline__ float big<float>() { return 3.0e38f; }
template <> __device__ __forceinline__ double big<double>() { return 1.0e300; }

// Parallel-segment threshold on a*e - b*b relative to a*e. FP64 follows the
// exact reading (1e-14); FP32 uses 2^-10 (sin^2 of about 1.8 degrees) and a
// conservative correction of the lower bound for pairs below it.
template <typename T> __device__ __forceinline__ T kappa();
template <> __device__ __forceinline__ float kappa<float>() { return 0.0009765625f; }
template <> __device__ __forceinline__ double kappa<double>() { return 1e-14; }

// Prepared triangle: vertices, unit normal and plane offset, inward edge
// normals g_k = n x e_k with offsets h_k = g_k . p_k (inside test of a
// projected point), squared edge lengths and their reciprocals.
// 32 scalars; the same order is used for the LDS copy.
template <typename T>
struct PTri {
    R3<T> p0, p1, p2;
    R3<T> n; T off;
    R3<T> g0; T h0;
    R3<T> g1; T h1;
    R3<T> g2; T h2;
    T ee0, ee1, ee2, ie0, ie1, ie2, emax;
};

template <typename T>
__device__ __forceinline__ PTri<T> prep(R3<T> p0, R3<T> p1, R3<T> p2)
{
    PTri<T> t;
    t.p0 = p0; t.p1 = p1; t.p2 = p2;
    R3<T> e0 = p1 - p0, e1 = p2 - p1, e2 = p0 - p2;
    R3<T> nn = cross(e0, p2 - p0);
    T inv = rsq(dot(nn, nn));
    t.n = nn * inv;
    t.off = dot(t.n, p0);
    t.g0 = cross(t.n, e0); t.h0 = dot(t.g0, p0);
    t.g1 = cross(t.n, e1); t.h1 = dot(t.g1, p1);
    t.g2 = cross(t.n, e2); t.h2 = dot(t.g2, p2);
    t.ee0 = dot(e0, e0); t.ee1 = dot(e1, e1); t.ee2 = dot(e2, e2);
    t.ie0 = recip(t.ee0); t.ie1 = recip(t.ee1); t.ie2 = recip(t.ee2);
    T m = t.ee0 > t.ee1 ? t.ee0 : t.ee1;
    m = m > t.ee2 ? m : t.ee2;
    t.emax = root(m);
    return t;
}

// Squared distance of a point to the face interior of B (big() when the
// projection falls outside); s receives the signed height over B's plane.
template <typename T>
__device__ __forceinline__ T vert_face(R3<T> x, const PTri<T>& B, T& s)
{
    s = dot(B.n, x) - B.off;
    bool in = (dot(B.g0, x) >= B.h0) & (dot(B.g1, x) >= B.h1) & (dot(B.g2, x) >= B.h2);
    return in ? s * s : big<T>();
}

// Segments pa + s ea and pb + t eb with s, t in [0,1]: the line solution for s
// (0 when parallel) clamped, t optimal for s, and when t leaves [0,1] it is
// clamped and s re-solved (the classic clamped closest-point construction).
template <typename T>
__device__ __forceinline__ T seg_seg(R3<T> pa, R3<T> ea, T aa, T ia, R3<T> pb, R3<T> eb, T ee,
                                     T ie, bool& near, T& s_out, T& t_out)
{
    R3<T> r = pa - pb;
    T b = dot(ea, eb), c = dot(ea, r), f = dot(eb, r);
    T den = aa * ee - b * b;
    near = !(den > kappa<T>() * aa * ee);
    T s = near ? T(0) : clamp01((b * f - c * ee) * recip(den));
    T t = (b * s + f) * ie;
    T tc = clamp01(t);
    s = (t == tc) ? s : clamp01((b * tc - c) * ia);
    s_out = s; t_out = tc;
    R3<T> dv = r + ea * s - eb * tc;
    return dot(dv, dv);
}

// Does edge p->q of one triangle meet the closed triangle B? op, oq: heights
// of p and q over B's plane. Endpoints within 1e-12 * l of the plane (l the
// largest of |p-b0|, |q-b0|, |b1-b0|, |b2-b0|) count as lying in it; that case
// is left to the distance features, which are zero for coplanar overlap.
__device__ __forceinline__ bool edge_meets(R3<double> p, R3<double> q, double op, double oq,
                                           const PTri<double>& B, R3<double>& x)
{
    if ((op > 0.0 && oq > 0.0) || (op < 0.0 && oq < 0.0)) return false;
    double l2 = dot(p - B.p0, p - B.p0);
    double t2 = dot(q - B.p0, q - B.p0); l2 = t2 > l2 ? t2 : l2;
    t2 = B.ee0; l2 = t2 > l2 ? t2 : l2;
    t2 = B.ee2; l2 = t2 > l2 ? t2 : l2;
    double hm2 = 1e-24 * l2;
    if (op * op <= hm2 && oq * oq <= hm2) return false;
    R3<double> d = q - p;
    double s1 = dot(d, cross(B.p0 - p, B.p1 - p));
    double s2 = dot(d, cross(B.p1 - p, B.p2 - p));
    double s3 = dot(d, cross(B.p2 - p, B.p0 - p));
    bool pos = (s1 >= 0.0) & (s2 >= 0.0) & (s3 >= 0.0);
    bool neg = (s1 <= 0.0) & (s2 <= 0.0) & (s3 <= 0.0);
    if (!(pos | neg)) return false;
    x = p + d * (op / (op - oq));
    return true;
}

// FP32 test whether edge p->q may meet triangle B, conservative against the
// FP64 decision: the edge must reach across B's plane within mu (op, oq: the
// heights of p and q), and the three signed volumes of the edge against B's
// edges must not have strictly mixed signs, each widened by eps (mu times a
// bound of the volumes' sensitivity to moving a vertex; the FP32 vertices
// and transform differ from the FP64 ones by far less than mu).
__device__ __forceinline__ bool edge_may_meet(R3<float> p, R3<float> q, float op, float oq,
                                              const PTri<float>& B, float mu, float eps)
{
    if ((op > mu && oq > mu) || (op < -mu && oq < -mu)) return false;
    const R3<float> d = q - p;
    const R3<float> u0 = B.p0 - p, u1 = B.p1 - p, u2 = B.p2 - p;
    const float s1 = dot(d, cross(u0, u1)), s2 = dot(d, cross(u1, u2)), s3 = dot(d, cross(u2, u0));
    return ((s1 >= -eps) & (s2 >= -eps) & (s3 >= -eps)) | ((s1 <= eps) & (s2 <= eps) & (s3 <= eps));
}

// FP32 filter: squared feature distance (vertex-face and edge-edge; no
// intersection test), whether an edge pair is near parallel, and whether the
// triangles may intersect (both reach across each other's plane within mu
// and some edge may meet the other triangle).
__device__ __forceinline__ float pair_filter(const PTri<float>& A, const PTri<float>& B, float mu,
                                             bool& np, bool& xs)
{
    float s, best;
    float sa0, sa1, sa2, sb0, sb1, sb2;
    best = vert_face(A.p0, B, sa0);
    best = fminf(best, vert_face(A.p1, B, sa1));
    best = fminf(best, vert_face(A.p2, B, sa2));
    best = fminf(best, vert_face(B.p0, A, sb0));
    best = fminf(best, vert_face(B.p1, A, sb1));
    best = fminf(best, vert_face(B.p2, A, sb2));
    R3<float> ea[3] = {A.p1 - A.p0, A.p2 - A.p1, A.p0 - A.p2};
    R3<float> eb[3] = {B.p1 - B.p0, B.p2 - B.p1, B.p0 - B.p2};
    R3<float> pa[3] = {A.p0, A.p1, A.p2};
    R3<float> pb[3] = {B.p0, B.p1, B.p2};
    float aa[3] = {A.ee0, A.ee1, A.ee2}, ia[3] = {A.ie0, A.ie1, A.ie2};
    float bb[3] = {B.ee0, B.ee1, B.ee2}, ib[3] = {B.ie0, B.ie1, B.ie2};
    bool anynp = false;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            bool nr; float ss, tt;
            float d2 = seg_seg(pa[k], ea[k], aa[k], ia[k], pb[l], eb[l], bb[l], ib[l], nr, ss, tt);
            best = fminf(best, d2);
            anynp |= nr;
        }
    np = anynp;
    float amin = fminf(sa0, fminf(sa1, sa2)), amax = fmaxf(sa0, fmaxf(sa1, sa2));
    float bmin = fminf(sb0, fminf(sb1, sb2)), bmax = fmaxf(sb0, fmaxf(sb1, sb2));
    xs = (amin <= mu) & (amax >= -mu) & (bmin <= mu) & (bmax >= -mu);
    if (xs) {
        // Only triangles whose bounding spheres overlap can intersect; for
        // them every vertex-to-vertex distance is at most U and every edge at
        // most D, which bounds a signed volume's change under vertex moves of
        // size mu by mu (U^2 + 2 D U).
        const float D = fmaxf(A.emax, B.emax);
        const float U = 2.5f * (A.emax + B.emax) + mu;
        const float eps = mu * (U * U + 2.f * D * U);
        xs = edge_may_meet(A.p0, A.p1, sa0, sa1, B, mu, eps) || edge_may_meet(A.p1, A.p2, sa1, sa2, B, mu, eps) ||
             edge_may_meet(A.p2, A.p0, sa2, sa0, B, mu, eps) || edge_may_meet(B.p0, B.p1, sb0, sb1, A, mu, eps) ||
             edge_may_meet(B.p1, B.p2, sb1, sb2, A, mu, eps) || edge_may_meet(B.p2, B.p0, sb2, sb0, A, mu, eps);
    }
    (void)s;
    return best;
}

// Exact FP64 squared distance. Optionally the winning feature: 0..5 edge meets
// triangle (A's edges then B's), 6..8 A's vertex to B's face, 9..11 B's vertex
// to A's face, 12..20 edge pair (3 k + l); first strictly smaller wins.
template <bool WANT_FEATURE>
__device__ __forceinline__ double pair_exact(const PTri<double>& A, const PTri<double>& B,
                                             int& feat, R3<double>& xhit)
{
    double sa[3], sb[3];
    R3<double> pa[3] = {A.p0, A.p1, A.p2};
    R3<double> pb[3] = {B.p0, B.p1, B.p2};
    double best = big<double>();
    int bf = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double d2 = vert_face(pa[k], B, sa[k]);
        if (WANT_FEATURE) { if (d2 < best) { best = d2; bf = 6 + k; } }
        else best = fmin(best, d2);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double d2 = vert_face(pb[k], A, sb[k]);
        if (WANT_FEATURE) { if (d2 < best) { best = d2; bf = 9 + k; } }
        else best = fmin(best, d2);
    }
    R3<double> ea[3] = {A.p1 - A.p0, A.p2 - A.p1, A.p0 - A.p2};
    R3<double> eb[3] = {B.p1 - B.p0, B.p2 - B.p1, B.p0 - B.p2};
    double aa[3] = {A.ee0, A.ee1, A.ee2}, ia[3] = {A.ie0, A.ie1, A.ie2};
    double bb[3] = {B.ee0, B.ee1, B.ee2}, ib[3] = {B.ie0, B.ie1, B.ie2};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            bool nr; double ss, tt;
            double d2 = seg_seg(pa[k], ea[k], aa[k], ia[k], pb[l], eb[l], bb[l], ib[l], nr, ss, tt);
            if (WANT_FEATURE) { if (d2 < best) { best = d2; bf = 12 + 3 * k + l; } }
            else best = fmin(best, d2);
        }
    // Intersection: both triangles must reach across each other's plane.
    double amin = fmin(sa[0], fmin(sa[1], sa[2])), amax = fmax(sa[0], fmax(sa[1], sa[2]));
    double bmin = fmin(sb[0], fmin(sb[1], sb[2])), bmax = fmax(sb[0], fmax(sb[1], sb[2]));
    if ((amin <= 0.0) & (amax >= 0.0) & (bmin <= 0.0) & (bmax >= 0.0)) {
        R3<double> x;
        bool hit = false;
        int hk = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!hit && edge_meets(pa[k], pa[(k + 1) % 3], sa[k], sa[(k + 1) % 3], B, x)) {
                hit = true; hk = k; xhit = x;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!hit && edge_meets(pb[k], pb[(k + 1) % 3], sb[k], sb[(k + 1) % 3], A, x)) {
                hit = true; hk = 3 + k; xhit = x;
            }
        }
        if (hit) { best = 0.0; bf = hk; }
    }
    feat = bf;
    return best;
}

// Closest points of the winning feature (FP64, in A's frame). The feature's
// operands are picked by selects (no run-time array index, which would put
// the triangles in scratch memory) and only that feature is evaluated: a
// vertex's projection onto the other plane, or one segment pair. (Evaluating
// all 15 features and selecting the result kept them all live: 76 registers
// spilled in the re-decision kernel instead of 44.)
template <typename V>
__device__ __forceinline__ V pick3(int k, V a, V b, V c)
{
    return k == 0 ? a : (k == 1 ? b : c);
}

__device__ __forceinline__ void feature_points(const PTri<double>& A, const PTri<double>& B, int f,
                                               R3<double> xhit, R3<double>& qa, R3<double>& qb)
{
    // 6..8: A's vertex over B's face; 9..11: B's vertex over A's face
    const bool vfa = f >= 6 && f <= 8, vfb = f >= 9 && f <= 11, edge = f >= 12;
    const int kv = vfa ? f - 6 : (vfb ? f - 9 : 0);
    const R3<double> x = vfa ? pick3(kv, A.p0, A.p1, A.p2) : pick3(kv, B.p0, B.p1, B.p2);
    const R3<double> n = vfa ? B.n : A.n;
    const double s = dot(n, x) - (vfa ? B.off : A.off);
    const R3<double> proj = x - n * s;
    // 12..20: edge k of A against edge l of B
    const int e = edge ? f - 12 : 0, k = e / 3, l = e - 3 * k;
    const R3<double> pk = pick3(k, A.p0, A.p1, A.p2), pl = pick3(l, B.p0, B.p1, B.p2);
    const R3<double> ea = pick3(k, A.p1, A.p2, A.p0) - pk, eb = pick3(l, B.p1, B.p2, B.p0) - pl;
    bool nr;
    double ss, tt;
    seg_seg(pk, ea, pick3(k, A.ee0, A.ee1, A.ee2), pick3(k, A.ie0, A.ie1, A.ie2), pl, eb,
            pick3(l, B.ee0, B.ee1, B.ee2), pick3(l, B.ie0, B.ie1, B.ie2), nr, ss, tt);
    // 0..5: an edge meets the other triangle at xhit
    qa = vfa ? x : (vfb ? proj : (edge ? pk + ea * ss : xhit));
    qb = vfa ? proj : (vfb ? x : (edge ? pl + eb * tt : xhit));
}

}  // namespace mcd
