// gfx950 kernels for collision time stamps (section 5: the case
// distinctions, narrowing and widening; motion from section 2: linear in
// position, spherical-linear in rotation, i.e. constant v and world-frame w).
//
// Per triangle pair the first time in [0, dt] with d <= delta is found by
// scanning S+1 equidistant samples; an interval [t_k, t_k+1] whose ends are
// both above delta can still hold a crossing unless the Lipschitz envelope
// (d_k + d_k+1 - L h)/2 stays above delta, in which case it is halved down to
// a width tol; a bracketed crossing is bisected to width tol and the in-contact
// end is returned. L bounds how fast any distance between the two rigid
// bodies can change.
//
// GPU split: (1) FP32 distances at t = 0 for the kept tile pairs select the
// triangle pairs that can come within delta during the step; (2) a persistent
// FP32 sampler gives each lane one triangle pair, skips intervals that the
// Lipschitz envelope proves clear (with the FP32 margin mu), and hands the
// first interval it cannot clear to (3) an FP64 end-game that runs the exact
// interval logic (sampling, halving, bisection) from there on. Intervals the
// sampler clears hold no time with d <= delta, so the end-game returns the
// same time as the plain scan over every interval. Per pair the earliest
// (time, i, j) wins through one 64-bit atomic minimum on lattice keys.
#include "mcd_internal.h"
#include "mcd_geom.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

// Rotation matrix and position at time t of a state (x, unit q, v, w):
// q(t) = exp(t w / 2) * q0, x(t) = x0 + v t.
__device__ __forceinline__ void pose(const double* s, double t, double* R, double* x)
{
    double qw = s[3], qx = s[4], qy = s[5], qz = s[6];
    const double wx = s[10], wy = s[11], wz = s[12];
    const double wn = sqrt(wx * wx + wy * wy + wz * wz);
    if (wn > 0.0 && t != 0.0) {
        const double h = 0.5 * wn * t;
        double sn, cs;
        sincos(h, &sn, &cs);
        const double sw = sn / wn;
        const double ew = cs, ex = sw * wx, ey = sw * wy, ez = sw * wz;
        const double rw = ew * qw - ex * qx - ey * qy - ez * qz;
        const double rx = ew * qx + ex * qw + ey * qz - ez * qy;
        const double ry = ew * qy - ex * qz + ey * qw + ez * qx;
        const double rz = ew * qz + ex * qy - ey * qx + ez * qw;
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
    x[0] = s[0] + s[7] * t;
    x[1] = s[1] + s[8] * t;
    x[2] = s[2] + s[9] * t;
}

// B's body frame into A's body frame at time t: X_A = M X_B + m.
__device__ __forceinline__ void rel_at(const PairDev& P, double t, double* M, double* m)
{
    double Ra[9], xa[3], Rb[9], xb[3];
    pose(P.st_a, t, Ra, xa);
    pose(P.st_b, t, Rb, xb);
    const double d0 = xb[0] - xa[0], d1 = xb[1] - xa[1], d2 = xb[2] - xa[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c] + Ra[6 + r] * Rb[6 + c];
        m[r] = Ra[r] * d0 + Ra[3 + r] * d1 + Ra[6 + r] * d2;
    }
}

__device__ __forceinline__ double sample_time(int k, double dt, int S)
{
    return __ddiv_rn(__dmul_rn((double)k, dt), (double)S);
}

// FP32 relative transforms at the S+1 sample times of every pair.
__global__ void k_toi_table(const PairDev* __restrict__ pairs, int32_t npairs, int32_t rows,
                            float* __restrict__ table)
{
    const int64_t n = (int64_t)npairs * rows;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / rows), k = (int)(i - (int64_t)p * rows);
        const PairDev& P = pairs[p];
        if (k > P.samples) continue;
        double M[9], m[3];
        rel_at(P, sample_time(k, P.dt, P.samples), M, m);
        float* o = table + (P.table0 + k) * 12;
#pragma unroll
        for (int j = 0; j < 9; ++j) o[j] = (float)M[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) o[9 + j] = (float)m[j];
    }
}

// Persistent FP32 sampler. A lane owns one triangle pair at a time and takes
// a new one from the queue when it finishes, so lanes stay busy however
// unevenly long the scans are. State per lane: the last evaluated sample
// (time ts, FP32 lower bound ds of the distance) and the next interval k.
__global__ __launch_bounds__(64) void k_toi_scan(const PairDev* __restrict__ pairs, TriStore S,
                                                 const float* __restrict__ table,
                                                 const Cand* __restrict__ scan,
                                                 const int32_t* __restrict__ scan_count,
                                                 int64_t scan_cap, int32_t* queue,
                                                 int32_t* pair_kub, Cand* __restrict__ eg,
                                                 int32_t* eg_count, int64_t eg_cap,
                                                 unsigned long long* sample_count)
{
    const int lane = lane_id();
    const int64_t n = min((int64_t)scan_count[0], scan_cap);
    bool active = false, drained = false;
    int pair = 0, sa = 0, sb = 0, k = 0, Sn = 1;
    int64_t table0 = 0;
    PTri<float> A;
    R3<float> b0{0, 0, 0}, b1{0, 0, 0}, b2{0, 0, 0};
    float ds = 0.f, ts = 0.f, mu = 0.f, delta = 0.f, L = 0.f, h = 1.f, corr = 0.f, slack = 0.f;
    unsigned long long evals = 0;
    for (;;) {
        bool fresh = false;
        if (!drained) {
            const bool need = !active;
            const uint64_t m = __ballot(need);
            if (m) {
                int base = 0;
                if (lane == 0) base = atomicAdd(queue, __popcll(m));
                base = __shfl(base, 0);
                const int64_t slot = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
                if ((int64_t)base + __popcll(m) > n) drained = true;
                if (need && slot < n) {
                    const Cand c = scan[slot];
                    pair = c.pair; sa = c.ta; sb = c.tb;
                    const PairDev& P = pairs[pair];
                    mu = P.mu; delta = (float)P.delta; L = (float)P.L; corr = P.corr;
                    Sn = P.samples; h = (float)(P.dt / P.samples); table0 = P.table0;
                    slack = 1e-6f * L * (float)P.dt;
                    R3<float> a0, a1, a2;
                    load_tri(S.v32, S.cap, sa, a0, a1, a2);
                    A = prep(a0, a1, a2);
                    load_tri(S.v32, S.cap, sb, b0, b1, b2);
                    ds = c.t; ts = 0.f; k = 0;
                    active = true;
                    fresh = true;
                }
            }
        }
        bool emit = false;
        int ek = 0;
        if (fresh && ds <= delta + mu + slack) { emit = true; ek = 0; active = false; }
        bool ev = false;
        int kk = 0;
        if (active) {
            if (!(L > 0.f)) {
                active = false;              // no relative motion: nothing changes after t = 0
            } else {
                float need_t = ts + (ds - mu - slack - delta) / L;
                float kf = floorf(fminf(need_t / h, 1.0e6f)) - 1.f;
                kk = max(k, (int)kf);
                const int kub = __atomic_load_n(&pair_kub[pair], __ATOMIC_RELAXED);
                if (kk >= Sn || kk >= kub) active = false;
                else ev = true;
            }
        }
        if (__ballot(ev)) {
            if (ev) {
                const float* T = table + (table0 + kk + 1) * 12;
                const PTri<float> B = prep(xform(T, T + 9, b0), xform(T, T + 9, b1), xform(T, T + 9, b2));
                bool np, xs;
                const float d2 = pair_filter(A, B, mu, np, xs);
                const float dub = sqrtf(d2);
                const float dlb = xs ? 0.f : fmaxf(0.f, dub - (np ? corr : 0.f));
                ++evals;
                const float t1 = (float)(kk + 1) * h;
                if (!xs && dub + mu + slack < delta) atomicMin(&pair_kub[pair], kk + 1);
                if (dlb <= delta + mu + slack ||
                    (ds + dlb - 2.f * (mu + slack) - L * (t1 - ts)) * 0.5f <= delta) {
                    emit = true; ek = kk; active = false;
                } else {
                    ds = dlb; ts = t1; k = kk + 1;
                    if (k >= Sn) active = false;
                }
            }
        }
        if (__ballot(emit)) {
            const int64_t slot = reserve(emit, eg_count);
            if (emit && slot < eg_cap) eg[slot] = Cand{pair, sa, sb, (float)ek};
        }
        if (drained && !__ballot(active)) break;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) evals += __shfl_xor(evals, o);
    if (lane == 0 && evals) atomicAdd(sample_count, evals);
}

struct Span {
    double lo, hi, dlo, dhi;
    int32_t clo, chi;
};

__device__ __forceinline__ double dist_at(const PairDev& P, const PTri<double>& A, R3<double> b0,
                                          R3<double> b1, R3<double> b2, double t)
{
    double M[9], m[3];
    rel_at(P, t, M, m);
    const PTri<double> B = prep(xform(M, m, b0), xform(M, m, b1), xform(M, m, b2));
    int f;
    R3<double> x;
    return sqrt(pair_exact<false>(A, B, f, x));
}

// FP64 end-game: the exact interval logic from the handed-over interval on.
// One lane per triangle pair; intervals that cannot beat the pair's current
// best key are skipped.
__global__ __launch_bounds__(64) void k_toi_endgame(const PairDev* __restrict__ pairs, TriStore S,
                                                    const Cand* __restrict__ eg,
                                                    const int32_t* __restrict__ eg_count,
                                                    int64_t eg_cap, uint64_t* pair_key,
                                                    ToiOut* __restrict__ out,
                                                    unsigned long long* diag, int from_zero)
{
    const int64_t n = min((int64_t)eg_count[0], eg_cap);
    unsigned long long evals = 0, grazes = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Cand c = eg[e];
        const PairDev& P = pairs[c.pair];
        R3<double> a0, a1, a2, b0, b1, b2;
        load_tri(S.v64, S.cap, c.ta, a0, a1, a2);
        load_tri(S.v64, S.cap, c.tb, b0, b1, b2);
        const PTri<double> A = prep(a0, a1, a2);
        const uint64_t ij = ((uint64_t)(uint32_t)S.orig[c.ta] << 16) | (uint32_t)S.orig[c.tb];
        const int k0 = from_zero ? 0 : (int)c.t;
        const int Sn = P.samples;
        const double dt = P.dt, tol = P.tol, L = P.L, delta = P.delta;
        uint64_t rkey = ~0ull;
        double rt = 0.0;
        double dl = dist_at(P, A, b0, b1, b2, sample_time(k0, dt, Sn));
        ++evals;
        bool stop = false;
        if (k0 == 0) {
            if (dl <= delta) { rkey = ij; rt = 0.0; stop = true; }
            else if (dl - delta > L * dt) stop = true;
        }
        for (int k = k0; k < Sn && !stop; ++k) {
            const uint64_t best = __atomic_load_n(&pair_key[c.pair], __ATOMIC_RELAXED);
            if ((best >> 32) < (((uint64_t)k << LATTICE_BITS) + 1)) break;
            const double t0 = sample_time(k, dt, Sn), t1 = sample_time(k + 1, dt, Sn);
            const double dr = dist_at(P, A, b0, b1, b2, t1);
            ++evals;
            Span st[32];
            int sp = 0;
            st[sp++] = Span{t0, t1, dl, dr, 0, 1 << LATTICE_BITS};
            while (sp > 0) {
                const Span s = st[--sp];
                if (s.dhi <= delta) {
                    double lo = s.lo, hi = s.hi;
                    int32_t clo = s.clo, chi = s.chi;
                    while (__dsub_rn(hi, lo) > tol) {
                        const double mid = __dmul_rn(__dadd_rn(lo, hi), 0.5);
                        const int32_t cm = (clo + chi) >> 1;
                        ++evals;
                        if (dist_at(P, A, b0, b1, b2, mid) <= delta) { hi = mid; chi = cm; }
                        else { lo = mid; clo = cm; }
                    }
                    rkey = ((((uint64_t)k << LATTICE_BITS) + (uint64_t)chi) << 32) | ij;
                    rt = hi;
                    stop = true;
                    break;
                }
                const double env = __dmul_rn(__dsub_rn(__dadd_rn(s.dlo, s.dhi),
                                                       __dmul_rn(L, __dsub_rn(s.hi, s.lo))), 0.5);
                if (env > delta) continue;
                if (__dsub_rn(s.hi, s.lo) <= tol) { ++grazes; continue; }
                const double mid = __dmul_rn(__dadd_rn(s.lo, s.hi), 0.5);
                const int32_t cm = (s.clo + s.chi) >> 1;
                const double dm = dist_at(P, A, b0, b1, b2, mid);
                ++evals;
                if (sp + 2 > 32) { ++grazes; continue; }   // depth is bounded by the lattice
                st[sp++] = Span{mid, s.hi, dm, s.dhi, cm, s.chi};
                st[sp++] = Span{s.lo, mid, s.dlo, dm, s.clo, cm};
            }
            dl = dr;
        }
        if (rkey != ~0ull) atomicMin((unsigned long long*)&pair_key[c.pair], (unsigned long long)rkey);
        out[e] = ToiOut{rkey, rt};
    }
    if (evals) atomicAdd(&diag[0], evals);
    if (grazes) atomicAdd(&diag[1], grazes);
}

// The double time of each pair's winning key.
__global__ void k_toi_final(const Cand* __restrict__ eg, const int32_t* __restrict__ eg_count,
                            int64_t eg_cap, const ToiOut* __restrict__ out,
                            const uint64_t* __restrict__ pair_key, double* pair_t)
{
    const int64_t n = min((int64_t)eg_count[0], eg_cap);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const ToiOut o = out[e];
        if (o.key != ~0ull && o.key == pair_key[eg[e].pair]) pair_t[eg[e].pair] = o.t;
    }
}

// Distance and closest points (world frame) of one given triangle pair per
// particle pair, at the pair's stored transform.
__global__ __launch_bounds__(64) void k_pair_eval(const PairDev* __restrict__ pairs, int32_t npairs,
                                                  TriStore S, const int32_t* __restrict__ ij,
                                                  PairOut* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const PairDev& P = pairs[p];
    const int io = ij[2 * p], jo = ij[2 * p + 1];
    PairOut r;
    r.toi = 0.0;
    r.status = 0;
    if (io < 0 || jo < 0) {
        r.d = __longlong_as_double(0x7ff0000000000000ll);
        r.pa[0] = r.pa[1] = r.pa[2] = r.pb[0] = r.pb[1] = r.pb[2] = 0.0;
        r.tri_a = r.tri_b = -1;
        r.contact = 0;
        out[p] = r;
        return;
    }
    const int64_t sa = S.pos[P.tri0_a + io], sb = S.pos[P.tri0_b + jo];
    R3<double> a0, a1, a2, b0, b1, b2;
    load_tri(S.v64, S.cap, sa, a0, a1, a2);
    load_tri(S.v64, S.cap, sb, b0, b1, b2);
    const PTri<double> A = prep(a0, a1, a2);
    const PTri<double> B = prep(xform(P.M, P.m, b0), xform(P.M, P.m, b1), xform(P.M, P.m, b2));
    int f;
    R3<double> xh, qa, qb;
    const double e2 = pair_exact<true>(A, B, f, xh);
    feature_points(A, B, f, xh, qa, qb);
    r.d = sqrt(e2);
    R3<double> wa = xform(P.Ra, P.xa, qa), wb = xform(P.Ra, P.xa, qb);
    r.pa[0] = wa.x; r.pa[1] = wa.y; r.pa[2] = wa.z;
    r.pb[0] = wb.x; r.pb[1] = wb.y; r.pb[2] = wb.z;
    r.tri_a = io;
    r.tri_b = jo;
    r.contact = e2 <= P.delta * P.delta ? 1 : 0;
    out[p] = r;
}

inline int blocks_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_toi_table(const Launch& L, const PairDev* pairs, int32_t npairs, int32_t rows,
                            float* table)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_toi_table, dim3(blocks_for((int64_t)npairs * rows, 128, 8192)), dim3(128), 0,
                       L.stream, pairs, npairs, rows, table);
    return hipGetLastError();
}

hipError_t launch_toi_scan(const Launch& L, const PairDev* pairs, const TriStore& S,
                           const float* table, const Cand* scan, const int32_t* scan_count,
                           int64_t scan_cap, int32_t* queue, int32_t* pair_kub, Cand* eg,
                           int32_t* eg_count, int64_t eg_cap, unsigned long long* sample_count,
                           int grid)
{
    hipLaunchKernelGGL(k_toi_scan, dim3(grid), dim3(64), 0, L.stream, pairs, S, table, scan,
                       scan_count, scan_cap, queue, pair_kub, eg, eg_count, eg_cap, sample_count);
    return hipGetLastError();
}

hipError_t launch_toi_endgame(const Launch& L, const PairDev* pairs, const TriStore& S,
                              const Cand* eg, const int32_t* eg_count, int64_t eg_cap,
                              uint64_t* pair_key, ToiOut* out, unsigned long long* diag,
                              int from_zero)
{
    hipLaunchKernelGGL(k_toi_endgame, dim3(blocks_for(eg_cap, 64, 4096)), dim3(64), 0, L.stream,
                       pairs, S, eg, eg_count, eg_cap, pair_key, out, diag, from_zero);
    return hipGetLastError();
}

hipError_t launch_toi_final(const Launch& L, const Cand* eg, const int32_t* eg_count,
                            int64_t eg_cap, const ToiOut* out, const uint64_t* pair_key,
                            double* pair_t)
{
    hipLaunchKernelGGL(k_toi_final, dim3(blocks_for(eg_cap, 256, 2048)), dim3(256), 0, L.stream, eg,
                       eg_count, eg_cap, out, pair_key, pair_t);
    return hipGetLastError();
}

hipError_t launch_pair_eval(const Launch& L, const PairDev* pairs, int32_t npairs,
                            const TriStore& S, const int32_t* ij, PairOut* out)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_eval, dim3((npairs + 63) / 64), dim3(64), 0, L.stream, pairs, npairs,
                       S, ij, out);
    return hipGetLastError();
}

}  // namespace mcd
