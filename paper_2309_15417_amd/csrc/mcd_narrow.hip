// gfx950 kernels of the paper's own collision-time estimate (section 5,
// "Collision time detection": narrowing). Rotation is neglected, as the paper
// does for this estimate: each triangle keeps its orientation at the start
// of the step and moves with its particle's velocity, so B moves relative to
// A by w = R_a^T (v_b - v_a) T over a span [0, T], in A's body frame. Per
// triangle pair, a round evaluates
//  - each of the 6 vertices against the other triangle at the start and the
//    end of the span and, when the vertex's path crosses the triangle's
//    plane inside the span, at the crossing;
//  - each of the 9 edge pairs at the start, the middle and the end;
// and the earliest evaluation time with distance <= delta is the pair's
// contact time. A round gives each particle pair the earliest contact time
// over its triangle pairs; while that is earlier than T it becomes T and the
// next round runs. One wave per tile pair (lane = A triangle, B's tile moved
// into A's frame in LDS); swept tile and triangle spheres skip what cannot
// come within delta during the span.
#include "mcd_internal.h"
#include "mcd_geom.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

// Squared distance of point x to triangle B: the height when the projection
// falls inside the face, else the nearest of the three edges.
__device__ __forceinline__ double point_tri2(R3<double> x, const PTri<double>& B)
{
    double h;
    double d2 = vert_face(x, B, h);
    const R3<double> p[3] = {B.p0, B.p1, B.p2};
    const double ee[3] = {B.ee0, B.ee1, B.ee2}, ie[3] = {B.ie0, B.ie1, B.ie2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R3<double> e = p[(k + 1) % 3] - p[k];
        const double s = clamp01(dot(x - p[k], e) * ie[k]);
        const R3<double> r = x - (p[k] + e * s);
        d2 = fmin(d2, dot(r, r));
        (void)ee[k];
    }
    return d2;
}

// Earliest fraction in {0, plane crossing, 1} at which x + s w is within
// delta of B (2: none).
__device__ __forceinline__ double vertex_time(R3<double> x, R3<double> w, const PTri<double>& B, double d2max)
{
    if (point_tri2(x, B) <= d2max) return 0.0;
    const double wn = dot(w, B.n);
    if (wn != 0.0) {
        const double s = -(dot(B.n, x) - B.off) / wn;
        if (s > 0.0 && s < 1.0 && point_tri2(x + w * s, B) <= d2max) return s;
    }
    return point_tri2(x + w, B) <= d2max ? 1.0 : 2.0;
}

// Earliest fraction in {0, 1/2, 1} at which edge (pa, ea) and edge (pb, eb)
// moved by s w are within delta (2: none).
__device__ __forceinline__ double edge_time(R3<double> pa, R3<double> ea, double aa, double ia, R3<double> pb,
                                            R3<double> eb, double bb, double ib, R3<double> w, double d2max)
{
    bool nr;
    double s, t;
    if (seg_seg(pa, ea, aa, ia, pb, eb, bb, ib, nr, s, t) <= d2max) return 0.0;
    if (seg_seg(pa, ea, aa, ia, pb + w * 0.5, eb, bb, ib, nr, s, t) <= d2max) return 0.5;
    if (seg_seg(pa, ea, aa, ia, pb + w, eb, bb, ib, nr, s, t) <= d2max) return 1.0;
    return 2.0;
}

__device__ double narrow_time(const PTri<double>& A, const PTri<double>& B, R3<double> w, double d2max)
{
    const R3<double> mw = w * -1.0;
    double best = 2.0;
    best = fmin(best, vertex_time(A.p0, mw, B, d2max));
    best = fmin(best, vertex_time(A.p1, mw, B, d2max));
    best = fmin(best, vertex_time(A.p2, mw, B, d2max));
    best = fmin(best, vertex_time(B.p0, w, A, d2max));
    best = fmin(best, vertex_time(B.p1, w, A, d2max));
    best = fmin(best, vertex_time(B.p2, w, A, d2max));
    const R3<double> pa[3] = {A.p0, A.p1, A.p2}, pb[3] = {B.p0, B.p1, B.p2};
    const R3<double> ea[3] = {A.p1 - A.p0, A.p2 - A.p1, A.p0 - A.p2};
    const R3<double> eb[3] = {B.p1 - B.p0, B.p2 - B.p1, B.p0 - B.p2};
    const double aa[3] = {A.ee0, A.ee1, A.ee2}, ia[3] = {A.ie0, A.ie1, A.ie2};
    const double bb[3] = {B.ee0, B.ee1, B.ee2}, ib[3] = {B.ie0, B.ie1, B.ie2};
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            best = fmin(best, edge_time(pa[k], ea[k], aa[k], ia[k], pb[l], eb[l], bb[l], ib[l], w, d2max));
    return best;
}

// Distance of the segment c + s w (s in [0, 1]) to point a.
__device__ __forceinline__ double sweep_gap(R3<double> c, R3<double> w, R3<double> a)
{
    const R3<double> d = c - a;
    const double ww = dot(w, w);
    const double s = ww > 0.0 ? clamp01(-dot(d, w) / ww) : 0.0;
    const R3<double> e = d + w * s;
    return sqrt(dot(e, e));
}

__device__ __forceinline__ R3<double> rel_motion(const PairDev& P, double T)
{
    // R_a^T (v_b - v_a) T: B's displacement relative to A, in A's frame
    const double dv[3] = {P.st_b[7] - P.st_a[7], P.st_b[8] - P.st_a[8], P.st_b[9] - P.st_a[9]};
    R3<double> w;
    w.x = (P.Ra[0] * dv[0] + P.Ra[3] * dv[1] + P.Ra[6] * dv[2]) * T;
    w.y = (P.Ra[1] * dv[0] + P.Ra[4] * dv[1] + P.Ra[7] * dv[2]) * T;
    w.z = (P.Ra[2] * dv[0] + P.Ra[5] * dv[1] + P.Ra[8] * dv[2]) * T;
    return w;
}

// One round over every tile pair. argmin = 0: each particle pair's earliest
// contact time into next (double bits, atomic minimum). argmin = 1: the
// triangle pairs whose contact time equals the pair's final time T put their
// caller (i, j) into ij (atomic minimum of i << 16 | j).
__global__ __launch_bounds__(64) void k_narrow_round(const PairDev* __restrict__ pairs, TriStore S,
                                                     const Item* __restrict__ items,
                                                     const int32_t* __restrict__ item_count, int64_t item_cap,
                                                     const double* __restrict__ pair_T, uint64_t* pair_next,
                                                     uint32_t* pair_ij, int argmin,
                                                     unsigned long long* eval_slots)
{
    __shared__ double sb[64 * 9];
    const int lane = lane_id();
    const int64_t n = min((int64_t)item_count[0], item_cap);
    unsigned long long nev = 0;
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const Item w_ = items[it];
        const PairDev& P = pairs[w_.pair];
        const double T = pair_T[w_.pair];
        if (!(T >= 0.0)) continue;
        const int ta = w_.tiles >> 16, tb = w_.tiles & 0xffff;
        const R3<double> w = rel_motion(P, T);
        const double reach = P.delta + 2.0 * (double)P.mu;
        // swept tile spheres
        const float4 ca = S.tile_sph[P.tile0_a + ta], cb = S.tile_sph[P.tile0_b + tb];
        const R3<double> cbA = xform(P.M, P.m, R3<double>{(double)cb.x, (double)cb.y, (double)cb.z});
        if (sweep_gap(cbA, w, R3<double>{(double)ca.x, (double)ca.y, (double)ca.z}) - (double)ca.w - (double)cb.w >
            reach)
            continue;
        const int nbt = min(TILE, P.nb - tb * TILE), nat = min(TILE, P.na - ta * TILE);
        // B's tile in A's frame, in LDS
        __syncthreads();
        if (lane < nbt) {
            R3<double> b0, b1, b2;
            load_tri_packed(S, (int64_t)P.tri0_b + tb * TILE + lane, b0, b1, b2);
            b0 = xform(P.M, P.m, b0); b1 = xform(P.M, P.m, b1); b2 = xform(P.M, P.m, b2);
            double* o = sb + 9 * lane;
            o[0] = b0.x; o[1] = b0.y; o[2] = b0.z; o[3] = b1.x; o[4] = b1.y; o[5] = b1.z;
            o[6] = b2.x; o[7] = b2.y; o[8] = b2.z;
        }
        __syncthreads();
        if (lane < nat) {
            const int64_t ia = (int64_t)P.tri0_a + ta * TILE + lane;
            R3<double> a0, a1, a2;
            load_tri_packed(S, ia, a0, a1, a2);
            const PTri<double> A = prep(a0, a1, a2);
            const float4 sa = S.tri_sph[ia];
            const R3<double> sac{(double)sa.x, (double)sa.y, (double)sa.z};
            const double d2max = P.delta * P.delta;
            double best = 2.0;
            uint32_t bij = 0xffffffffu;
            for (int j = 0; j < nbt; ++j) {
                const float4 sbj = S.tri_sph[P.tri0_b + tb * TILE + j];
                const R3<double> cj = xform(P.M, P.m, R3<double>{(double)sbj.x, (double)sbj.y, (double)sbj.z});
                if (sweep_gap(cj, w, sac) - (double)sa.w - (double)sbj.w > reach) continue;
                const double* o = sb + 9 * j;
                const PTri<double> B = prep(R3<double>{o[0], o[1], o[2]}, R3<double>{o[3], o[4], o[5]},
                                            R3<double>{o[6], o[7], o[8]});
                const double s = narrow_time(A, B, w, d2max);
                ++nev;
                if (!argmin) {
                    best = fmin(best, s);
                } else if (s <= 1.0 && s * T == T) {
                    const uint32_t key = ((uint32_t)S.orig[ia] << 16) |
                                         (uint32_t)S.orig[(int64_t)P.tri0_b + tb * TILE + j];
                    bij = min(bij, key);
                }
            }
            if (!argmin && best <= 1.0) {
                const double t = best * T;
                atomicMin((unsigned long long*)&pair_next[w_.pair], (unsigned long long)__double_as_longlong(t));
            }
            if (argmin && bij != 0xffffffffu) atomicMin(&pair_ij[w_.pair], bij);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nev += __shfl_xor(nev, o);
    put_wave_stat(eval_slots, nev);
}

__global__ void k_narrow_init(const int32_t* nq, int32_t ncap, const PairDev* __restrict__ pairs, double* pair_T,
                              uint64_t* pair_next, uint32_t* pair_ij, int32_t* found)
{
    const int n = min(nq[0], ncap);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        pair_T[p] = pairs[p].dt;
        pair_next[p] = ~0ull;
        pair_ij[p] = 0xffffffffu;
        found[p] = 0;
    }
}

// After a round: a pair whose earliest contact is before its span's end
// narrows the span to it (and the rounds continue).
__global__ void k_narrow_update(const int32_t* nq, int32_t ncap, double* pair_T, uint64_t* pair_next,
                                int32_t* found, int32_t* changed)
{
    const int n = min(nq[0], ncap);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint64_t nx = pair_next[p];
        if (nx == ~0ull) continue;
        found[p] = 1;
        const double t = __longlong_as_double((long long)nx);
        if (t < pair_T[p]) {
            pair_T[p] = t;
            *changed = 1;
        }
        pair_next[p] = ~0ull;
    }
}

inline int grid_of(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_narrow_init(const Launch& L, const int32_t* nq, int32_t ncap, const PairDev* pairs,
                              double* pair_T, uint64_t* pair_next, uint32_t* pair_ij, int32_t* found)
{
    if (ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow_init, dim3(grid_of(ncap, 256, 1024)), dim3(256), 0, L.stream, nq, ncap, pairs,
                       pair_T, pair_next, pair_ij, found);
    return hipGetLastError();
}

hipError_t launch_narrow_round(const Launch& L, const PairDev* pairs, const TriStore& S, const Item* items,
                               const int32_t* item_count, int64_t item_cap, const double* pair_T,
                               uint64_t* pair_next, uint32_t* pair_ij, int argmin, unsigned long long* eval_slots,
                               int grid)
{
    hipLaunchKernelGGL(k_narrow_round, dim3(grid), dim3(64), 0, L.stream, pairs, S, items, item_count, item_cap,
                       pair_T, pair_next, pair_ij, argmin, eval_slots);
    return hipGetLastError();
}

hipError_t launch_narrow_update(const Launch& L, const int32_t* nq, int32_t ncap, double* pair_T,
                                uint64_t* pair_next, int32_t* found, int32_t* changed)
{
    if (ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow_update, dim3(grid_of(ncap, 256, 1024)), dim3(256), 0, L.stream, nq, ncap, pair_T,
                       pair_next, found, changed);
    return hipGetLastError();
}

}  // namespace mcd
