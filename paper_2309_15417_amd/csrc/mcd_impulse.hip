// Particle interaction (section 6): the impulses exchanged at the contact
// points of a cluster, by a Picard iteration that updates the contribution
// of one contact point at a time, on a colouring of the contact graph so
// that the contacts of one colour (no two share a particle) update in
// parallel.
//
// Clusters (the connected components of the contact graph) are independent:
// one workgroup solves each, per sweep the cluster's colours in turn with the
// contacts of a colour spread over its threads and a barrier between colours,
// until the cluster's own convergence.
// Per contact (normal n from particle a to b, contact point X): the
// separation speed u_n of the two material points at X is driven to its
// target max(0, -e u_n0) by a non-negative normal impulse (Gauss-Seidel with
// projection), then a Coulomb tangential impulse opposes the sliding
// velocity within the cone |l_t| <= mu l_n; each update moves an impulse a
// fraction relax of the way. The iteration ends after the first sweep whose
// largest change of a contact's impulse is at most tol times the largest
// impulse, or after max_iter sweeps.
#include "mcd_internal.h"

namespace mcd {
namespace {

struct Vec {
    double x, y, z;
};
__device__ __forceinline__ Vec vmake(const double* p) { return Vec{p[0], p[1], p[2]}; }
__device__ __forceinline__ void vstore(double* p, Vec a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
__device__ __forceinline__ Vec operator+(Vec a, Vec b) { return Vec{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ Vec operator-(Vec a, Vec b) { return Vec{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Vec operator*(Vec a, double s) { return Vec{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double vdot(Vec a, Vec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Vec vcross(Vec a, Vec b)
{
    return Vec{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ Vec mul3(const double* M, Vec a)
{
    return Vec{M[0] * a.x + M[1] * a.y + M[2] * a.z, M[3] * a.x + M[4] * a.y + M[5] * a.z,
               M[6] * a.x + M[7] * a.y + M[8] * a.z};
}

// Velocity of the material point at lever arm r = X - centre of body b, an
// impulse J applied there, and d . ((Iinv (r x d)) x r), the rotational share
// of the effective inverse mass along d.
__device__ __forceinline__ Vec arm_vel(const ImpBody& b, Vec r) { return vmake(b.vc) + vcross(vmake(b.w), r); }
__device__ __forceinline__ void arm_apply(ImpBody& b, Vec r, Vec J)
{
    vstore(b.vc, vmake(b.vc) + J * b.invm);
    vstore(b.w, vmake(b.w) + mul3(b.Iinv, vcross(r, J)));
}
__device__ __forceinline__ double arm_share(const ImpBody& b, Vec r, Vec d)
{
    return vdot(d, vcross(mul3(b.Iinv, vcross(r, d)), r));
}

__device__ __forceinline__ double block_max(double v, double* red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double m = red[0];
    for (int k = 1; k < nw; ++k) m = fmax(m, red[k]);
    return m;
}

// Bodies: centre of mass and velocities in the world frame, world-frame
// inverse inertia R Ib^-1 R'.
__global__ void k_imp_bodies(int32_t np, const double* __restrict__ state, const double* __restrict__ mprop,
                             ImpBody* bodies)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const double* s = state + 13 * i;
        const double* mp = mprop + 13 * i;   // mass, centre (3), inertia about it (9)
        double qw = s[3], qx = s[4], qy = s[5], qz = s[6];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                             2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                             2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
        ImpBody b;
        b.invm = 1.0 / mp[0];
        const Vec rc = mul3(R, vmake(mp + 1));
        const Vec w = vmake(s + 10);
        vstore(b.rc, rc);
        vstore(b.xc, vmake(s) + rc);
        vstore(b.w, w);
        vstore(b.vc, vmake(s + 7) + vcross(w, rc));
        // inverse of the body inertia (symmetric positive definite) by cofactors
        const double* I = mp + 4;
        const double c00 = I[4] * I[8] - I[5] * I[7], c01 = I[5] * I[6] - I[3] * I[8], c02 = I[3] * I[7] - I[4] * I[6];
        const double det = I[0] * c00 + I[1] * c01 + I[2] * c02;
        const double Bi[9] = {c00 / det, (I[2] * I[7] - I[1] * I[8]) / det, (I[1] * I[5] - I[2] * I[4]) / det,
                              c01 / det, (I[0] * I[8] - I[2] * I[6]) / det, (I[2] * I[3] - I[0] * I[5]) / det,
                              c02 / det, (I[1] * I[6] - I[0] * I[7]) / det, (I[0] * I[4] - I[1] * I[3]) / det};
        double T[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Bi[3 * r + k] * R[3 * c + k];
                T[3 * r + c] = acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * r + k] * T[3 * k + c];
                b.Iinv[3 * r + c] = acc;
            }
        bodies[i] = b;
    }
}

// One cluster per workgroup: its contacts are con[cl.c0 .. cl.c1) in colour
// order, colour k spanning col_off[cl.off + k .. cl.off + k + 1); its bodies
// are bodies[cl.b0 .. cl.b0 + cl.nb), kept in LDS when there are at most
// IMP_LDS_BODIES of them.
__global__ __launch_bounds__(IMP_THREADS) void k_imp_solve(ImpBody* bodies, const ImpContact* __restrict__ con,
                                                           const ImpCluster* __restrict__ clusters,
                                                           const int32_t* __restrict__ col_off, ImpOpts o,
                                                           ImpWork* work, double* __restrict__ impulse,
                                                           int32_t* sweeps)
{
    __shared__ double red[IMP_THREADS / 64];
    __shared__ ImpBody lbody[IMP_LDS_BODIES];
    const int tid = threadIdx.x, nt = blockDim.x;
    const ImpCluster cl = clusters[blockIdx.x];
    const int nc = cl.c1 - cl.c0;
    const bool in_lds = cl.nb <= IMP_LDS_BODIES;
    ImpBody* bd = in_lds ? lbody : bodies + cl.b0;
    ImpWork* wk = work + cl.c0;
    if (in_lds)
        for (int i = tid; i < cl.nb; i += nt) lbody[i] = bodies[cl.b0 + i];
    __syncthreads();
    // contacts: normal (pb - pa, or between the centres when the closest
    // points coincide), lever arms from the contact point, normal effective
    // inverse mass and the separation-speed target max(0, -e u_n0)
    for (int r = tid; r < nc; r += nt) {
        const ImpContact& k = con[cl.c0 + r];
        const ImpBody &A = bd[k.a], &B = bd[k.b];
        const Vec p = vmake(k.pa), q = vmake(k.pb);
        const Vec X = (p + q) * 0.5;
        const Vec dv = q - p;
        const double d = sqrt(vdot(dv, dv));
        Vec n;
        if (d > 0.0) {
            n = dv * (1.0 / d);
        } else {
            const Vec e = vmake(B.xc) - vmake(A.xc);
            const double de = sqrt(vdot(e, e));
            n = de > 0.0 ? e * (1.0 / de) : Vec{0.0, 0.0, 1.0};
        }
        const Vec ra = X - vmake(A.xc), rb = X - vmake(B.xc);
        ImpWork w;
        vstore(w.n, n);
        vstore(w.ra, ra);
        vstore(w.rb, rb);
        w.kn = A.invm + B.invm + arm_share(A, ra, n) + arm_share(B, rb, n);
        w.target = fmax(0.0, -o.restitution * vdot(arm_vel(B, rb) - arm_vel(A, ra), n));
        w.ln = 0.0;
        w.lt[0] = w.lt[1] = w.lt[2] = 0.0;
        wk[r] = w;
    }
    __syncthreads();
    int it = 0;
    while (it < o.max_iter) {
        ++it;
        double maxd = 0.0;
        for (int k = 0; k < cl.ncol; ++k) {
            const int e0 = col_off[cl.off + k] - cl.c0, e1 = col_off[cl.off + k + 1] - cl.c0;
            for (int r = e0 + tid; r < e1; r += nt) {
                const ImpContact& ct = con[cl.c0 + r];
                ImpWork& w = wk[r];
                ImpBody &A = bd[ct.a], &B = bd[ct.b];
                const Vec n = vmake(w.n), ra = vmake(w.ra), rb = vmake(w.rb);
                const double un = vdot(arm_vel(B, rb) - arm_vel(A, ra), n);
                const double star = fmax(0.0, w.ln + (w.target - un) / w.kn);
                const double nl = w.ln + o.relax * (star - w.ln);
                const double dl = nl - w.ln;
                w.ln = nl;
                arm_apply(B, rb, n * dl);
                arm_apply(A, ra, n * (-dl));
                double change = fabs(dl);
                if (o.friction > 0.0) {
                    const Vec u = arm_vel(B, rb) - arm_vel(A, ra);
                    const Vec ut = u - n * vdot(u, n);
                    const double s = sqrt(vdot(ut, ut));
                    const Vec lt = vmake(w.lt);
                    Vec trial = lt;
                    if (s > 0.0) {
                        const Vec t = ut * (1.0 / s);
                        const double kt = A.invm + B.invm + arm_share(A, ra, t) + arm_share(B, rb, t);
                        trial = lt - ut * (1.0 / kt);
                    }
                    const double cap = o.friction * w.ln, tl = sqrt(vdot(trial, trial));
                    if (tl > cap && tl > 0.0) trial = trial * (cap / tl);
                    const Vec nlt = lt + (trial - lt) * o.relax;
                    const Vec dlt = nlt - lt;
                    vstore(w.lt, nlt);
                    arm_apply(B, rb, dlt);
                    arm_apply(A, ra, dlt * -1.0);
                    change += sqrt(vdot(dlt, dlt));
                }
                maxd = fmax(maxd, change);
            }
            __syncthreads();
        }
        double maxl = 0.0;
        for (int r = tid; r < nc; r += nt)
            maxl = fmax(maxl, wk[r].ln + sqrt(wk[r].lt[0] * wk[r].lt[0] + wk[r].lt[1] * wk[r].lt[1] +
                                                wk[r].lt[2] * wk[r].lt[2]));
        maxd = block_max(maxd, red);
        maxl = block_max(maxl, red);
        if (maxd <= o.tol * maxl) break;
    }
    if (in_lds)
        for (int i = tid; i < cl.nb; i += nt) bodies[cl.b0 + i] = lbody[i];
    for (int r = tid; r < nc; r += nt) {
        double* out = impulse + 4 * con[cl.c0 + r].idx;
        out[0] = wk[r].ln;
        out[1] = wk[r].lt[0];
        out[2] = wk[r].lt[1];
        out[3] = wk[r].lt[2];
    }
    if (tid == 0) sweeps[blockIdx.x] = it;
}

// New state velocities: the origin's velocity from the centre's, written at
// each body's slot in the caller's particle order.
__global__ void k_imp_vel(int32_t np, const ImpBody* __restrict__ bodies, const int32_t* __restrict__ slot,
                          double* __restrict__ vel)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const ImpBody& b = bodies[i];
        const Vec w = vmake(b.w);
        double* out = vel + 6 * slot[i];
        vstore(out, vmake(b.vc) - vcross(w, vmake(b.rc)));
        vstore(out + 3, w);
    }
}

}  // namespace

hipError_t launch_impulse(const Launch& L, int32_t np, const double* state, const double* mprop, ImpBody* bodies,
                          const ImpContact* con, int32_t ncl, const ImpCluster* clusters, const int32_t* col_off,
                          const ImpOpts& o, ImpWork* work, double* impulse, const int32_t* vel_slot, double* vel,
                          int32_t* sweeps)
{
    const int gb = (np + 255) / 256;
    hipLaunchKernelGGL(k_imp_bodies, dim3(gb), dim3(256), 0, L.stream, np, state, mprop, bodies);
    hipLaunchKernelGGL(k_imp_solve, dim3(ncl), dim3(IMP_THREADS), 0, L.stream, bodies, con, clusters, col_off, o,
                       work, impulse, sweeps);
    hipLaunchKernelGGL(k_imp_vel, dim3(gb), dim3(256), 0, L.stream, np, bodies, vel_slot, vel);
    return hipGetLastError();
}

}  // namespace mcd
