// gfx950 kernels of the broad phase inside a set of particles (section 3 of
// the paper): check 1, the space-time bounding boxes (each particle's
// bounding sphere plus halo at the start and at the end of the step, boxed
// together), then check 2, the space-time tubes (the spheres moving linearly
// over the step come within reach of each other at some common time); and
// the identification of the unconnected subgraphs (clusters) by repeated
// min-labelling until nothing changes.
//
// The member list holds one or more segments (the cluster queries of a
// batch); pairs are formed inside a segment only, one wave per member row,
// so a row's pairs come out in member order and rows in member order: the
// list is ordered by (position of a, position of b) within each segment.
#include "mcd_internal.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

__global__ __launch_bounds__(256) void k_bp_prep(const int32_t* __restrict__ hdr, const int32_t* __restrict__ pid,
                                                 int32_t cap, const int32_t* __restrict__ seg_off, int32_t seg_cap,
                                                 const PartDev* __restrict__ parts, int32_t npart,
                                                 const MeshDev* __restrict__ meshes, int32_t nmesh, double dt,
                                                 BpMember* __restrict__ out, int32_t* counters, int err_word)
{
    const int m = min(hdr[0], cap);
    const int nseg = min(hdr[1], seg_cap);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        BpMember b;
        memset(&b, 0, sizeof b);
        // the segment holding member i: the last offset not above i
        int lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (seg_off[mid] <= i) lo = mid; else hi = mid;
        }
        b.end = seg_off[lo + 1];
        const int id = pid[i];
        b.pid = id;
        int err = 0;
        if (id < 0 || id >= npart || parts[id].mesh < 0 || parts[id].mesh >= nmesh) err = GATHER_BAD_ID;
        else if (!meshes[parts[id].mesh].alive) err = GATHER_DEAD_MESH;
        if (err) {
            atomicOr(&counters[err_word], err);
        } else {
            const PartDev& P = parts[id];
            const MeshDev& M = meshes[P.mesh];
            b.r = M.radius + M.halo;
            for (int c = 0; c < 3; ++c) {
                b.x[c] = P.s[c];
                b.v[c] = P.s[7 + c];
                const double x1 = P.s[c] + P.s[7 + c] * dt;
                b.lo[c] = fmin(P.s[c], x1) - b.r;
                b.hi[c] = fmax(P.s[c], x1) + b.r;
            }
            b.valid = 1;
        }
        out[i] = b;
    }
}

// Check 1 and check 2 for members a and b.
__device__ __forceinline__ bool bp_keep(const BpMember& a, const BpMember& b, double dt)
{
    if (!b.valid) return false;
    // check 1: the space-time boxes overlap
    for (int c = 0; c < 3; ++c)
        if (a.lo[c] > b.hi[c] || b.lo[c] > a.hi[c]) return false;
    // check 2: the closest approach of the two centres over [0, dt]
    double d[3], dv[3], vv = 0.0, dvx = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = b.x[c] - a.x[c];
        dv[c] = b.v[c] - a.v[c];
        vv += dv[c] * dv[c];
        dvx += d[c] * dv[c];
    }
    double t = 0.0;
    if (dt > 0.0 && vv > 0.0) t = fmin(dt, fmax(0.0, -dvx / vv));
    double r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double e = d[c] + dv[c] * t;
        r2 += e * e;
    }
    const double lim = a.r + b.r;
    return r2 <= lim * lim;
}

// One wave per member row: count (write = 0) or write (write = 1) the row's
// pairs with the later members of its segment, in member order.
__global__ __launch_bounds__(64) void k_bp_rows(const int32_t* __restrict__ hdr, int32_t cap,
                                                const BpMember* __restrict__ mem, double dt, int write,
                                                int32_t* __restrict__ row_cnt, const int64_t* __restrict__ row_off,
                                                int32_t* __restrict__ pairs_out, int32_t* __restrict__ pos_out,
                                                int64_t pair_cap)
{
    const int m = min(hdr[0], cap);
    const int lane = lane_id();
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const BpMember a = mem[i];
        int cnt = 0;
        const int64_t base = write ? row_off[i] : 0;
        if (a.valid) {
            for (int j0 = i + 1; j0 < a.end; j0 += 64) {
                const int j = j0 + lane;
                bool keep = false;
                int pj = 0;
                if (j < a.end) {
                    const BpMember b = mem[j];
                    keep = bp_keep(a, b, dt);
                    pj = b.pid;
                }
                const uint64_t bits = __ballot(keep);
                if (write && keep) {
                    const int64_t slot = base + cnt + __popcll(bits & ((1ull << lane) - 1ull));
                    if (slot < pair_cap) {
                        pairs_out[2 * slot] = a.pid;
                        pairs_out[2 * slot + 1] = pj;
                        if (pos_out) { pos_out[2 * slot] = i; pos_out[2 * slot + 1] = j; }
                    }
                }
                cnt += __popcll(bits);
            }
        }
        if (!write && lane == 0) row_cnt[i] = cnt;
    }
}

// Exclusive scan of the row counts (one block): row offsets, the pair total
// into the list header (0 when it exceeds the capacity, with the overflow
// bit set) and the 64-bit counter c64[total_at], and each segment's first
// pair into seg_pairs[0..nseg] (seg_pairs[nseg] = total).
__global__ __launch_bounds__(1024) void k_bp_scan(const int32_t* __restrict__ hdr, int32_t cap,
                                                  const int32_t* __restrict__ row_cnt, int64_t* __restrict__ row_off,
                                                  const int32_t* __restrict__ seg_off, int32_t seg_cap,
                                                  int64_t* __restrict__ seg_pairs, int32_t* hdr_list,
                                                  int64_t pair_cap, int32_t* counters, int err_word, int total_at)
{
    const int m = min(hdr[0], cap);
    const int nseg = min(hdr[1], seg_cap);
    __shared__ long long wsum[16];
    __shared__ long long total;
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int seg = (m + 1023) / 1024;
    const int lo = min(tid * seg, m), hi = min(lo + seg, m);
    long long sum = 0;
    for (int i = lo; i < hi; ++i) sum += row_cnt[i];
    long long x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    long long run = x - sum;
    for (int q = 0; q < wv; ++q) run += wsum[q];
    for (int i = lo; i < hi; ++i) { row_off[i] = run; run += row_cnt[i]; }
    if (tid == 1023) total = run;
    __syncthreads();
    for (int s = tid; s <= nseg; s += 1024) {
        const int r = seg_off[s];
        seg_pairs[s] = (s == nseg || r >= m) ? total : row_off[r];
    }
    if (tid == 0) {
        ((unsigned long long*)counters)[total_at] = (unsigned long long)total;
        if (total > pair_cap) {
            atomicOr(&counters[err_word], (int)GATHER_OVERFLOW);
            hdr_list[0] = 0;
        } else {
            hdr_list[0] = (int32_t)total;
        }
    }
}

__global__ void k_label_init(int32_t* label, int32_t m)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) label[i] = i;
}

// One sweep of min-labelling over the pair graph: each edge lowers the
// larger label of its ends to the smaller; *changed is set when a label fell.
__global__ void k_label_sweep(const int32_t* __restrict__ pos, int64_t npairs, int32_t* label, int32_t* changed)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < npairs;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int a = pos[2 * k], b = pos[2 * k + 1];
        const int la = label[a], lb = label[b];
        if (la < lb) {
            if (atomicMin(&label[b], la) > la) *changed = 1;
        } else if (lb < la) {
            if (atomicMin(&label[a], lb) > lb) *changed = 1;
        }
    }
}

inline int grid_of(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_broad_phase(const Launch& L, const int32_t* hdr, const int32_t* pid, int32_t cap,
                              const int32_t* seg_off, int32_t seg_cap, const PartDev* parts, int32_t npart,
                              const MeshDev* meshes, int32_t nmesh, double dt, BpMember* mem, int32_t* row_cnt,
                              int64_t* row_off, int64_t* seg_pairs, int32_t* hdr_list, int32_t* pairs_out,
                              int32_t* pos_out, int64_t pair_cap, int32_t* counters, int err_word, int total_at)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bp_prep, dim3(grid_of(cap, 256, 1024)), dim3(256), 0, L.stream, hdr, pid, cap, seg_off,
                       seg_cap, parts, npart, meshes, nmesh, dt, mem, counters, err_word);
    const int rows = grid_of(cap, 1, L.num_cu * 32);
    hipLaunchKernelGGL(k_bp_rows, dim3(rows), dim3(64), 0, L.stream, hdr, cap, mem, dt, 0, row_cnt, row_off,
                       pairs_out, pos_out, pair_cap);
    hipLaunchKernelGGL(k_bp_scan, dim3(1), dim3(1024), 0, L.stream, hdr, cap, row_cnt, row_off, seg_off, seg_cap,
                       seg_pairs, hdr_list, pair_cap, counters, err_word, total_at);
    hipLaunchKernelGGL(k_bp_rows, dim3(rows), dim3(64), 0, L.stream, hdr, cap, mem, dt, 1, row_cnt, row_off,
                       pairs_out, pos_out, pair_cap);
    return hipGetLastError();
}

hipError_t launch_label_init(const Launch& L, int32_t* label, int32_t m)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_init, dim3(grid_of(m, 256, 1024)), dim3(256), 0, L.stream, label, m);
    return hipGetLastError();
}

hipError_t launch_label_sweep(const Launch& L, const int32_t* pos, int64_t npairs, int32_t* label, int32_t* changed)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_sweep, dim3(grid_of(npairs, 256, 4096)), dim3(256), 0, L.stream, pos, npairs, label,
                       changed);
    return hipGetLastError();
}

}  // namespace mcd
