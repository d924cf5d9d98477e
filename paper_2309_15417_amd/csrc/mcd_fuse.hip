// gfx950 kernels of contact fusion (section 5, after the contact-point
// definition: contact points close in space are fused into one, which also
// centres them within parallel triangles). Per particle pair, over its
// contact records in (tri_a, tri_b) order: the first record not yet in a
// group seeds one, and every later free record whose contact point (the
// midpoint of its closest points) lies within the pair's threshold delta of
// the seed's joins it. A group becomes one record: the seed's triangles, the
// mean of its members' contact points, and the distance vector of its member
// nearest to contact (lowest position on ties), so that the record's
// midpoint is the mean and |p_b - p_a| its distance; `merged` counts the
// members. One wave per pair; the groups are written in place at the start
// of the pair's segment, then compacted.
#include "mcd_internal.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

__device__ __forceinline__ void midpoint(const mcd_contact& c, double* x)
{
    x[0] = 0.5 * (c.pa[0] + c.pb[0]);
    x[1] = 0.5 * (c.pa[1] + c.pb[1]);
    x[2] = 0.5 * (c.pa[2] + c.pb[2]);
}

__global__ __launch_bounds__(64) void k_fuse(const PairDev* __restrict__ pairs, const int32_t* nq,
                                             const int32_t* __restrict__ off, mcd_contact* rec,
                                             int32_t* __restrict__ grp, int32_t* __restrict__ ngroups)
{
    const int n = nq[0];
    const int lane = lane_id();
    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int o0 = off[p], m = off[p + 1] - o0;
        const double r2 = pairs[p].delta * pairs[p].delta;
        for (int k = lane; k < m; k += 64) grp[o0 + k] = -1;
        __syncthreads();
        int g = 0, from = 0;
        for (;;) {
            // the first free record at or after `from`
            int seed = -1;
            for (int k0 = from; k0 < m && seed < 0; k0 += 64) {
                const int k = k0 + lane;
                const uint64_t free_ = __ballot(k < m && grp[o0 + k] < 0);
                if (free_) seed = k0 + (int)__ffsll((long long)free_) - 1;
            }
            if (seed < 0) break;
            const mcd_contact s = rec[o0 + seed];
            double xs[3];
            midpoint(s, xs);
            // members: the seed and the later free records within delta
            double sx = 0.0, sy = 0.0, sz = 0.0;
            double dbest = 1e300;
            int kbest = 0x7fffffff, cnt = 0;
            for (int k0 = seed; k0 < m; k0 += 64) {
                const int k = k0 + lane;
                bool in = false;
                mcd_contact c;
                double x[3] = {0.0, 0.0, 0.0};
                if (k < m && grp[o0 + k] < 0) {
                    c = rec[o0 + k];
                    midpoint(c, x);
                    const double dx = x[0] - xs[0], dy = x[1] - xs[1], dz = x[2] - xs[2];
                    in = k == seed || dx * dx + dy * dy + dz * dz <= r2;
                }
                if (in) {
                    grp[o0 + k] = g;
                    sx += x[0]; sy += x[1]; sz += x[2];
                    ++cnt;
                    if (c.d < dbest || (c.d == dbest && k < kbest)) { dbest = c.d; kbest = k; }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                sx += __shfl_xor(sx, o);
                sy += __shfl_xor(sy, o);
                sz += __shfl_xor(sz, o);
                cnt += __shfl_xor(cnt, o);
                const double od = __shfl_xor(dbest, o);
                const int ok = __shfl_xor(kbest, o);
                if (od < dbest || (od == dbest && ok < kbest)) { dbest = od; kbest = ok; }
            }
            const mcd_contact b = rec[o0 + kbest];
            __syncthreads();   // every lane has read the records before one is overwritten
            if (lane == 0) {
                mcd_contact f = s;
                const double inv = 1.0 / cnt;
                const double mx[3] = {sx * inv, sy * inv, sz * inv};
                for (int c = 0; c < 3; ++c) {
                    const double h = 0.5 * (b.pb[c] - b.pa[c]);
                    f.pa[c] = mx[c] - h;
                    f.pb[c] = mx[c] + h;
                }
                f.d = b.d;
                f.merged = cnt;
                rec[o0 + g] = f;
            }
            __syncthreads();
            ++g;
            from = seed + 1;
        }
        if (lane == 0) ngroups[p] = g;
    }
}

__global__ void k_fuse_gather(const int32_t* nq, const int32_t* __restrict__ off, const int32_t* __restrict__ goff,
                              const mcd_contact* __restrict__ rec, mcd_contact* __restrict__ out)
{
    const int n = nq[0];
    for (int p = blockIdx.x; p < n; p += gridDim.x) {
        const int g = goff[p + 1] - goff[p];
        for (int k = threadIdx.x; k < g; k += blockDim.x) out[goff[p] + k] = rec[off[p] + k];
    }
}

}  // namespace

hipError_t launch_fuse(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t npairs, const int32_t* off,
                       mcd_contact* rec, int32_t* grp, int32_t* ngroups)
{
    if (npairs <= 0) return hipSuccess;
    const int grid = npairs < L.num_cu * 16 ? npairs : L.num_cu * 16;
    hipLaunchKernelGGL(k_fuse, dim3(grid), dim3(64), 0, L.stream, pairs, nq, off, rec, grp, ngroups);
    return hipGetLastError();
}

hipError_t launch_fuse_gather(const Launch& L, const int32_t* nq, int32_t npairs, const int32_t* off,
                              const int32_t* goff, const mcd_contact* rec, mcd_contact* out)
{
    if (npairs <= 0) return hipSuccess;
    const int grid = npairs < L.num_cu * 16 ? npairs : L.num_cu * 16;
    hipLaunchKernelGGL(k_fuse_gather, dim3(grid), dim3(64), 0, L.stream, nq, off, goff, rec, out);
    return hipGetLastError();
}

}  // namespace mcd
