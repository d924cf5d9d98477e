// gfx950 kernels for the static contact query (section 5: geometric model and
// contact points). One 64-lane wave owns one work item = (A tile, B tile) of a
// particle pair: lane l holds A's triangle l in registers, B's tile is
// transformed into A's body frame once and staged in LDS, and every lane then
// walks the 64 B triangles through LDS broadcast reads. Work items are popped
// from a device counter by a persistent grid, so uneven meshes balance.
#include <rocprim/device/device_radix_sort.hpp>

#include "mcd_internal.h"
#include "mcd_geom.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Sums each slot row of the plan into its 64-bit counter: block (t, part)
// adds part `part` of row t (STAT_PARTS parts), one atomic per block.
constexpr int STAT_PARTS = 16;

__global__ __launch_bounds__(256) void k_stat_reduce(const uint64_t* __restrict__ slots, StatPlan plan,
                                                     unsigned long long* counters64)
{
    __shared__ unsigned long long part[4];
    const int t = blockIdx.x / STAT_PARTS, pi = blockIdx.x % STAT_PARTS;
    if (t >= plan.n) return;
    const int w = plan.waves[t];
    const int lo = (int)((int64_t)w * pi / STAT_PARTS), hi = (int)((int64_t)w * (pi + 1) / STAT_PARTS);
    const uint64_t* row = slots + (int64_t)t * STAT_WAVES;
    unsigned long long v = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) v += row[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) part[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long sum = part[0] + part[1] + part[2] + part[3];
        if (sum) atomicAdd(&counters64[plan.dst[t]], sum);   // rows may share a counter
    }
}

// Pair preparation (section 2: relative moving frame; section 5: halo and
// step bound), one thread per pair, in FP64. Poses of both particles at the
// pair's time t (rotation about the rotation centre by exp(t w / 2) q0,
// position x0 + v t); the transform of B's body frame into A's, M = Ra^T Rb,
// m = Ra^T (xb - xa); the contact threshold delta = eps_a + eps_b; the
// coordinate scale |m| + (relative travel) + R_a + R_b that sets the FP32
// margin mu; for time stamps the motion bound L = |v_a - v_b| + |w_a| R_a +
// |w_b| R_b of every distance between the two bodies and the motion reach
// L dt that widens the cull thresholds. Every field of the record is written.
__global__ __launch_bounds__(128) void k_pair_prep(const int32_t* __restrict__ hdr_src,
                                                   const PairSrc* __restrict__ src, int32_t ncap,
                                                   PrepOpts o, int32_t* __restrict__ hdr_dst,
                                                   PairDev* __restrict__ out,
                                                   const uint64_t* __restrict__ tkey,
                                                   const double* __restrict__ tval, int tmode)
{
    const int n = min(hdr_src[0], ncap);
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) hdr_dst[0] = n;
    for (int i = tid; i < n; i += gridDim.x * blockDim.x) {
        const PairSrc& Q = src[i];
        PairDev& P = out[i];
        double sa[13], sb[13];
#pragma unroll
        for (int k = 0; k < 13; ++k) { sa[k] = Q.sa[k]; sb[k] = Q.sb[k]; }
        double t = Q.t;
        bool empty = false;
        if (tkey) {
            // contacts at the pair's time stamp (none: no tile pairs)
            const uint64_t key = tkey[i];
            empty = key == ~0ull;
            t = (empty || (key >> 32) == 0) ? 0.0 : tval[i];
            if (tmode & PREP_ZERO_SPIN)
                for (int k = 10; k < 13; ++k) sa[k] = sb[k] = 0.0;
        }
        double Ra[9], Rb[9], xa[3], xb[3], M[9], m[3];
        pose(sa, t, Ra, xa);
        pose(sb, t, Rb, xb);
        const double dx = xb[0] - xa[0], dy = xb[1] - xa[1], dz = xb[2] - xa[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) M[3 * r + c] = Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c] + Ra[6 + r] * Rb[6 + c];
            m[r] = Ra[r] * dx + Ra[3 + r] * dy + Ra[6 + r] * dz;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) { P.M[k] = M[k]; P.Ra[k] = Ra[k]; P.Mf[k] = (float)M[k]; }
#pragma unroll
        for (int k = 0; k < 3; ++k) { P.m[k] = m[k]; P.xa[k] = xa[k]; P.mf[k] = (float)m[k]; }
        P.tri0_a = Q.tri0_a; P.tri0_b = Q.tri0_b;
        P.na = Q.na; P.nb = Q.nb;
        P.tile0_a = Q.tile0_a; P.tile0_b = Q.tile0_b;
        P.nta = Q.nta; P.ntb = Q.ntb;
        P.group0_a = Q.group0_a; P.group0_b = Q.group0_b;
        const double delta = Q.halo_a + Q.halo_b;
        const double dist = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        const bool toi = o.dt > 0.0 && t == 0.0;
        double L = 0.0, travel = 0.0, vr = 0.0, wa = 0.0, wb = 0.0;
        if (toi) {
            const double v0 = sa[7] - sb[7], v1 = sa[8] - sb[8], v2 = sa[9] - sb[9];
            vr = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            wa = sqrt(sa[10] * sa[10] + sa[11] * sa[11] + sa[12] * sa[12]);
            wb = sqrt(sb[10] * sb[10] + sb[11] * sb[11] + sb[12] * sb[12]);
            L = vr + wa * Q.rad_a + wb * Q.rad_b;
            travel = vr * o.dt;
        }
        P.vr = (float)vr;
        P.wa = (float)wa;
        P.wb = (float)wb;
        const double lam = dist + travel + Q.rad_a + Q.rad_b;
        const double mu = o.margin_c * 0x1p-23 * lam;
        const double emax = fmax(Q.emax_a, Q.emax_b);
        const double corr = 0.03125 * emax;   // sqrt(2^-10) times the longest edge
        const double reach = toi ? L * o.dt * (1.0 + 1e-6) : 0.0;
        P.delta = delta;
        P.mu = (float)mu;
        P.corr = (float)corr;
        P.mu64 = 1e-9 * lam;
        P.corr64 = 1e-7 * emax;
        P.thr2 = (float)((delta + mu + reach) * (delta + mu + reach));
        P.thr2_np = (float)((delta + mu + corr + reach) * (delta + mu + corr + reach));
        P.cull = (float)(delta + mu + reach);
        P.flags = o.flags;
        P.dt = toi ? o.dt : 0.0;
        P.L = L;
        P.tol = toi ? o.tol_rel * o.dt : 0.0;
        P.samples = toi ? o.samples : 0;
#pragma unroll
        for (int k = 0; k < 13; ++k) { P.st_a[k] = toi ? sa[k] : 0.0; P.st_b[k] = toi ? sb[k] : 0.0; }
        P.table0 = Q.table0;
        P.tp0 = (tmode & PREP_TP0_WORDS) ? Q.tp0 / 64 + i : Q.tp0;
        if (empty) P.na = P.nb = P.nta = P.ntb = 0;
    }
}

// Pair sources gathered on the device from a device pair list: what the host
// staging copies per pair (both state snapshots, both meshes' records, list
// offsets), read from the device copies of the particle and mesh tables.
// Pass 1: one thread per pair writes its source record and its offset count;
// pass 2 (one block) scans the counts into tp0, checks the totals against the
// capacities and empties every pair if they do not fit.
__global__ __launch_bounds__(256) void k_pair_gather(const int32_t* __restrict__ nlist,
                                                     const int32_t* __restrict__ dlist, int32_t ncap,
                                                     const PartDev* __restrict__ parts, int32_t npart,
                                                     const MeshDev* __restrict__ meshes, int32_t nmesh,
                                                     double t, int toi, int32_t rows,
                                                     int32_t* __restrict__ hdr_src, PairSrc* __restrict__ src,
                                                     int64_t* __restrict__ cnt, int32_t* counters, int err_word)
{
    const int n = min(nlist[0], ncap);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) hdr_src[0] = n;
    if (i >= n) return;
    const int ia = dlist[2 * i], ib = dlist[2 * i + 1];
    int err = 0;
    const PartDev* A = nullptr;
    const PartDev* B = nullptr;
    if (ia < 0 || ib < 0 || ia >= npart || ib >= npart) err = GATHER_BAD_ID;
    else {
        A = &parts[ia];
        B = &parts[ib];
        if (A->mesh < 0 || B->mesh < 0 || A->mesh >= nmesh || B->mesh >= nmesh) err = GATHER_BAD_ID;
        else if (ia == ib) err = GATHER_SAME;
        else if (!meshes[A->mesh].alive || !meshes[B->mesh].alive) err = GATHER_DEAD_MESH;
    }
    PairSrc Q;
    memset(&Q, 0, sizeof Q);
    Q.t = t;
    if (!err) {
        const MeshDev ma = meshes[A->mesh], mb = meshes[B->mesh];
#pragma unroll
        for (int k = 0; k < 13; ++k) { Q.sa[k] = A->s[k]; Q.sb[k] = B->s[k]; }
        Q.halo_a = ma.halo; Q.halo_b = mb.halo;
        Q.rad_a = ma.radius; Q.rad_b = mb.radius;
        Q.emax_a = ma.emax; Q.emax_b = mb.emax;
        Q.tri0_a = ma.tri0; Q.tri0_b = mb.tri0;
        Q.na = ma.nt; Q.nb = mb.nt;
        Q.tile0_a = ma.tile0; Q.tile0_b = mb.tile0;
        Q.nta = ma.ntile; Q.ntb = mb.ntile;
        Q.group0_a = ma.group0; Q.group0_b = mb.group0;
    } else {
        // an empty pair: unit quaternions, no tiles
        Q.sa[3] = Q.sb[3] = 1.0;
        atomicOr(&counters[err_word], err);
    }
    Q.table0 = toi ? (int64_t)i * rows : 0;
    const int64_t tp = (int64_t)Q.nta * Q.ntb;
    cnt[i] = tp;
    cnt[n + i] = (int64_t)Q.na * Q.nb;
    src[i] = Q;
}

__global__ __launch_bounds__(1024) void k_pair_offsets(const int32_t* __restrict__ nlist, int32_t ncap, int toi,
                                                       int64_t item_cap, int64_t word_cap,
                                                       PairSrc* __restrict__ src, const int64_t* __restrict__ cnt,
                                                       int32_t* counters, int err_word, int words_at, int tiles_at,
                                                       int tris_at)
{
    const int n = min(nlist[0], ncap);
    __shared__ long long wsum[16], wtiles[16], wtris[16];
    __shared__ int overflow;
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int seg = (n + 1023) / 1024;
    const int lo = min(tid * seg, n), hi = min(lo + seg, n);
    long long sum = 0, tiles = 0, tris = 0;
    for (int i = lo; i < hi; ++i) {
        const long long tp = cnt[i];
        sum += toi ? tp : (tp + 63) / 64;
        tiles += tp;
        tris += cnt[n + i];
    }
    long long x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tiles += __shfl_xor(tiles, o);
        tris += __shfl_xor(tris, o);
    }
    if (lane == 63) wsum[wv] = x;
    if (lane == 0) { wtiles[wv] = tiles; wtris[wv] = tris; }
    __syncthreads();
    if (tid == 0) {
        long long tw = 0, tt = 0, tr = 0;
        for (int q = 0; q < 16; ++q) { tw += wsum[q]; tt += wtiles[q]; tr += wtris[q]; }
        unsigned long long* c64 = (unsigned long long*)counters;
        c64[words_at] = (unsigned long long)tw;
        c64[tiles_at] = (unsigned long long)tt;
        c64[tris_at] = (unsigned long long)tr;
        overflow = (tt > item_cap || tw > word_cap) ? 1 : 0;
        if (overflow) atomicOr(&counters[err_word], (int)GATHER_OVERFLOW);
    }
    __syncthreads();
    long long run = x - sum;
    for (int q = 0; q < wv; ++q) run += wsum[q];
    for (int i = lo; i < hi; ++i) {
        const long long tp = cnt[i];
        src[i].tp0 = run;
        run += toi ? tp : (tp + 63) / 64;
        if (overflow) { src[i].nta = src[i].ntb = 0; src[i].na = src[i].nb = 0; }
    }
}

// Device particle table update: records scattered to their ids.
__global__ void k_part_scatter(const int32_t* __restrict__ ids, const PartDev* __restrict__ recs, int32_t n,
                               PartDev* __restrict__ table)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        table[ids[i]] = recs[i];
}

// Start of a static query: zero the counters, reset the per-pair minima.
__global__ void k_init_static(uint32_t* counters, int ncounters, uint32_t* pair_ub, uint64_t* pair_d2,
                              uint64_t* pair_tie, int32_t* pair_cnt, int32_t npairs)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npairs || i < ncounters;
         i += gridDim.x * blockDim.x) {
        if (i < ncounters) counters[i] = 0u;
        if (i < npairs) { pair_ub[i] = 0xffffffffu; pair_d2[i] = ~0ull; pair_tie[i] = ~0ull; pair_cnt[i] = 0; }
    }
}

// Tile-pair cull: keep (tile_a, tile_b) when the bounding spheres (B's moved
// into A's frame) are within the pair's threshold. Three passes and no
// shared counter: k_cull_count counts each pair's kept tile pairs (one block
// per pair, grid-stride), k_cull_scan turns the counts into offsets in one
// block, and k_cull_write reads the count pass's bitmask and writes each
// pair's items contiguously at its offset.
__device__ __forceinline__ bool tile_keep(const PairDev& P, const TriStore& S, int dense, int ta, int tb)
{
    if (dense) return true;
    const float4 a = S.tile_sph[P.tile0_a + ta];
    const float4 b = S.tile_sph[P.tile0_b + tb];
    const R3<float> c = xform(P.Mf, P.mf, R3<float>{b.x, b.y, b.z});
    const float dx = c.x - a.x, dy = c.y - a.y, dz = c.z - a.z;
    const float gap = fsqrt(dx * dx + dy * dy + dz * dz) - a.w - b.w;
    return gap <= P.cull;
}

// The tile test on spheres staged in LDS: A's sphere, and B's with its
// centre already moved into A's frame (the same arithmetic as tile_keep).
__device__ __forceinline__ bool tile_keep_staged(const PairDev& P, float4 a, float4 c)
{
    const float dx = c.x - a.x, dy = c.y - a.y, dz = c.z - a.z;
    const float gap = fsqrt(dx * dx + dy * dy + dz * dz) - a.w - c.w;
    return gap <= P.cull;
}

// Tile spheres of a pair staged in LDS by the cull passes when both meshes
// have at most this many tiles (larger meshes read them from the store).
constexpr int CULL_TILES_LDS = 128;

// Group level (the coarser surrogate of a mesh: GROUP consecutive tiles in
// Morton order under one sphere holding their spheres): a group pair whose
// spheres are beyond the threshold holds no kept tile pair. The group test
// is widened by the margin mu against FP32 rounding, so it never drops a
// tile pair the tile test keeps.
__device__ __forceinline__ bool group_keep(const PairDev& P, const TriStore& S, int ga, int gb)
{
    const float4 a = S.grp_sph[P.group0_a + ga];
    const float4 b = S.grp_sph[P.group0_b + gb];
    const R3<float> c = xform(P.Mf, P.mf, R3<float>{b.x, b.y, b.z});
    const float dx = c.x - a.x, dy = c.y - a.y, dz = c.z - a.z;
    const float gap = fsqrt(dx * dx + dy * dy + dz * dz) - a.w - b.w;
    return gap <= P.cull + P.mu;
}

// Pairs with up to CULL_MASK_WORDS * 64 tile pairs build their bitmask in
// LDS; larger pairs set the bits in the (cleared) global words directly.
constexpr int CULL_MASK_WORDS = 512;
constexpr int CULL_GROUP_BATCH = 256;   // group pairs tested per round, one per thread

__global__ __launch_bounds__(256) void k_cull_count(const PairDev* __restrict__ pairs, const int32_t* nq,
                                                    int32_t ncap, TriStore S, int dense,
                                                    int32_t* __restrict__ pcount, int64_t* __restrict__ ptiled,
                                                    uint64_t* __restrict__ mask, unsigned long long* test_slots)
{
    const int npairs = min(nq[0], ncap);
    __shared__ int32_t wc[4];
    __shared__ unsigned long long wt[4], wn[4];
    __shared__ unsigned long long smask[CULL_MASK_WORDS];
    __shared__ int32_t glist[CULL_GROUP_BATCH];
    __shared__ int32_t gcount;
    __shared__ float4 tsa[CULL_TILES_LDS], tsb[CULL_TILES_LDS];
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    unsigned long long tests = 0;   // this thread's sphere tests (both levels)
    for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
        const PairDev& P = pairs[p];
        const int ntb = P.ntb, ntot = P.nta * ntb;
        int cnt = 0;
        unsigned long long tiled = 0;
        if (!dense) {
            // Two levels. Each round tests up to 256 group pairs, one per
            // thread, and lists the kept ones in LDS; then a wave takes a kept
            // group pair at a time, one lane per tile pair of its 8 x 8, and
            // each row of 8 decisions is ORed into the pair's mask words.
            const int nwords = (ntot + 63) / 64;
            const bool in_lds = nwords <= CULL_MASK_WORDS;
            unsigned long long* gm = (unsigned long long*)(mask + P.tp0);
            unsigned long long* mw = in_lds ? smask : gm;
            for (int w = tid; w < nwords; w += 256) mw[w] = 0ull;
            // both meshes' tile spheres in LDS (B's moved into A's frame), so
            // that each kept group pair's tests wait on no global load
            const bool staged = P.nta <= CULL_TILES_LDS && ntb <= CULL_TILES_LDS;
            if (staged) {
                if (tid < P.nta) tsa[tid] = S.tile_sph[P.tile0_a + tid];
                if (tid < ntb) {
                    const float4 b = S.tile_sph[P.tile0_b + tid];
                    const R3<float> c = xform(P.Mf, P.mf, R3<float>{b.x, b.y, b.z});
                    tsb[tid] = make_float4(c.x, c.y, c.z, b.w);
                }
            }
            const int nga = (P.nta + GROUP - 1) / GROUP, ngb = (ntb + GROUP - 1) / GROUP;
            const int ngp = nga * ngb;
            for (int g0 = 0; g0 < ngp; g0 += CULL_GROUP_BATCH) {
                if (tid == 0) gcount = 0;
                __syncthreads();   // also orders the cleared words before the ORs
                const int g = g0 + tid;
                if (g < ngp) {
                    // a pair of single-group meshes has nothing to skip at the
                    // group level: its one group pair is kept untested
                    const bool keep = ngp == 1 || (++tests, group_keep(P, S, g / ngb, g % ngb));
                    if (keep) glist[atomicAdd(&gcount, 1)] = g;
                }
                __syncthreads();
                const int ng = gcount;
                for (int e = wv; e < ng; e += 4) {
                    const int ge = glist[e];
                    const int ga = ge / ngb, gb = ge - ga * ngb;
                    const int ta = ga * GROUP + (lane >> 3), tb = gb * GROUP + (lane & 7);
                    bool keep = false;
                    if (ta < P.nta && tb < ntb) {
                        ++tests;
                        keep = staged ? tile_keep_staged(P, tsa[ta], tsb[tb]) : tile_keep(P, S, 0, ta, tb);
                        if (keep) {
                            ++cnt;
                            tiled += (unsigned long long)(min(TILE, P.na - ta * TILE) * min(TILE, P.nb - tb * TILE));
                        }
                    }
                    const uint64_t bal = __ballot(keep);
                    const unsigned long long row = (bal >> (lane & ~7)) & 0xffull;
                    if ((lane & 7) == 0 && row) {
                        // bits ta * ntb + gb * 8 + (0..7): may straddle two words
                        const int q = ta * ntb + gb * GROUP, w = q >> 6, sh = q & 63;
                        atomicOr(&mw[w], row << sh);
                        if (sh > 64 - GROUP) atomicOr(&mw[w + 1], row >> (64 - sh));
                    }
                }
                __syncthreads();
            }
            if (in_lds)
                for (int w = tid; w < nwords; w += 256) gm[w] = smask[w];
        }
        for (int k0 = 0; dense && k0 < ntot; k0 += 256) {
            const int k = k0 + tid;
            bool keep = false;
            if (k < ntot) {
                const int ta = k / ntb, tb = k - ta * ntb;
                keep = tile_keep(P, S, dense, ta, tb);
                if (keep) {
                    ++cnt;
                    tiled += (unsigned long long)(min(TILE, P.na - ta * TILE) * min(TILE, P.nb - tb * TILE));
                }
            }
            // the decisions, one bit per tile pair, for the write pass
            const uint64_t bits = __ballot(keep);
            if (lane == 0 && k0 + 64 * wv < ntot) mask[P.tp0 + (k0 >> 6) + wv] = bits;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            cnt += __shfl_xor(cnt, o);
            tiled += __shfl_xor(tiled, o);
        }
        if (lane == 0) { wc[wv] = cnt; wt[wv] = tiled; }
        __syncthreads();
        if (tid == 0) {
            pcount[p] = wc[0] + wc[1] + wc[2] + wc[3];
            ptiled[p] = (int64_t)(wt[0] + wt[1] + wt[2] + wt[3]);
        }
        __syncthreads();
    }
    if (test_slots) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o);
        if (lane == 0) wn[wv] = tests;
        __syncthreads();
        if (tid == 0) test_slots[blockIdx.x] = wn[0] + wn[1] + wn[2] + wn[3];
    }
}

// Exclusive scan of the per-pair counts in one block of 1024 threads (each
// thread a contiguous segment of pairs); the total is the item count.
__global__ __launch_bounds__(1024) void k_cull_scan(const int32_t* __restrict__ pcount,
                                                    const int64_t* __restrict__ ptiled, const int32_t* nq,
                                                    int32_t ncap, int32_t* __restrict__ poff,
                                                    int32_t* item_count, unsigned long long* tiled_total)
{
    const int npairs = min(nq[0], ncap);
    __shared__ int32_t wtot[16];
    __shared__ unsigned long long wtl[16];
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int seg = (npairs + 1023) / 1024;
    const int lo = min(tid * seg, npairs), hi = min(lo + seg, npairs);
    int sum = 0;
    unsigned long long tl = 0;
    for (int i = lo; i < hi; ++i) { sum += pcount[i]; tl += (unsigned long long)ptiled[i]; }
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tl += __shfl_xor(tl, o);
    if (lane == 63) wtot[wv] = x;
    if (lane == 0) wtl[wv] = tl;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wv; ++q) before += wtot[q];
    int run = before + x - sum;
    for (int i = lo; i < hi; ++i) { poff[i] = run; run += pcount[i]; }
    if (tid == 1023) item_count[0] = run;
    if (tid == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < 16; ++q) t += wtl[q];
        tiled_total[0] = t;
    }
}

// Write pass: every kept tile pair of a pair, in (tile_a, tile_b) order from
// the pair's offset on. The pair's mask words are staged in LDS, up to
// CULL_WRITE_WORDS at a time, with the exclusive scan of their bit counts;
// each thread then places its tile pairs by itself (its word's offset plus
// the kept bits below it in the word), so a large pair costs no barrier per
// chunk of tile pairs.
constexpr int CULL_WRITE_WORDS = 256;   // one per thread

__global__ __launch_bounds__(256) void k_cull_write(const PairDev* __restrict__ pairs, const int32_t* nq,
                                                    int32_t ncap, TriStore S, const int32_t* __restrict__ poff,
                                                    const uint64_t* __restrict__ mask, int dense,
                                                    Item* __restrict__ items, NearItem* __restrict__ nitems,
                                                    int64_t item_cap)
{
    const int npairs = min(nq[0], ncap);
    __shared__ unsigned long long wmask[CULL_WRITE_WORDS];
    __shared__ int32_t woff[CULL_WRITE_WORDS];
    __shared__ int32_t wtot[4];
    __shared__ float4 tcb[CULL_TILES_LDS];
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
        const PairDev& P = pairs[p];
        const int ntb = P.ntb, ntot = P.nta * ntb;
        const int nwords = (ntot + 63) / 64;
        int64_t base = poff[p];
        // B's tile centres in A's frame with radius plus reach, once per pair
        // (ordered before their use by the first barrier below)
        const float reach = (float)P.delta + P.mu * 2.f;
        const bool staged = !dense && ntb <= CULL_TILES_LDS;
        if (staged && tid < ntb) {
            const float4 bt = S.tile_sph[P.tile0_b + tid];
            const R3<float> cb = xform(P.Mf, P.mf, R3<float>{bt.x, bt.y, bt.z});
            tcb[tid] = make_float4(cb.x, cb.y, cb.z, bt.w + reach);
        }
        for (int w0 = 0; w0 < nwords; w0 += CULL_WRITE_WORDS) {
            const int w = w0 + tid;
            const unsigned long long m = w < nwords ? mask[P.tp0 + w] : 0ull;
            const int c = __popcll(m);
            int x = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) wtot[wv] = x;
            wmask[tid] = m;
            __syncthreads();
            int before = 0;
            for (int q = 0; q < wv; ++q) before += wtot[q];
            woff[tid] = before + x - c;
            const int round_total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
            __syncthreads();
            const int k_end = min(ntot, (w0 + CULL_WRITE_WORDS) * 64);
            for (int k = w0 * 64 + tid; k < k_end; k += 256) {
                const int lw = (k >> 6) - w0, b = k & 63;
                const unsigned long long mw = wmask[lw];
                if (!((mw >> b) & 1ull)) continue;
                const int64_t slot = base + woff[lw] + __popcll(mw & ((1ull << b) - 1ull));
                if (slot >= item_cap) continue;
                const int ta = k / ntb, tb = k - ta * ntb;
                if (dense) {
                    items[slot] = Item{p, (ta << 16) | tb};
                } else {
                    // B's tile centre in A's frame and the reach of the near-list
                    // test, so that the row test of k_near needs no pair record
                    float4 cb4;
                    if (staged) {
                        cb4 = tcb[tb];
                    } else {
                        const float4 bt = S.tile_sph[P.tile0_b + tb];
                        const R3<float> cb = xform(P.Mf, P.mf, R3<float>{bt.x, bt.y, bt.z});
                        cb4 = make_float4(cb.x, cb.y, cb.z, bt.w + reach);
                    }
                    nitems[slot] = NearItem{p, (ta << 16) | tb, P.tri0_a + ta * TILE, min(TILE, P.na - ta * TILE), cb4};
                }
            }
            base += round_total;
            __syncthreads();   // the next round's words replace these
        }
    }
}

// Dense queries (every pair's exact minimum, beyond the halo too): one wave
// per work item, lane = A triangle, B's tile moved into A's frame and
// prepared once in LDS, every triangle pair of the item evaluated.
//
// FP32 filter: triangle pairs that may be within delta (FP32 distance <=
// delta + mu, or possibly intersecting) are appended for the FP64
// re-decision; each item also records the smallest FP32 feature distance (an
// upper bound of the true minimum within mu) and a lower bound of the true
// minimum; per pair the smallest upper bound is kept for the FP64 refinement.
__global__ __launch_bounds__(64) void k_dist32(const PairDev* __restrict__ pairs, TriStore S,
                                               const Item* __restrict__ items,
                                               const int32_t* __restrict__ item_count,
                                               int64_t item_cap, PartialF* __restrict__ part,
                                               uint32_t* pair_ub, Cand* __restrict__ cands,
                                               int32_t* cand_count, int64_t cand_cap,
                                               int32_t* queue, unsigned long long* eval_slots)
{
    __shared__ float4 lds[TILE * F32_STRIDE];
    const int lane = lane_id();
    const int64_t nitems = min((int64_t)item_count[0], item_cap);
    unsigned long long nev = 0;
    int qbase = 0, qk = 4;
    for (;;) {
        const int it = pop_chunked<4>(queue, qbase, qk);
        if (it >= nitems) break;
        const Item w = items[it];
        const PairDev& P = pairs[w.pair];
        const int ta = w.tiles >> 16, tb = w.tiles & 0xffff;
        const int ia = ta * TILE + lane;
        const bool a_ok = ia < P.na;
        const int nbt = min(TILE, P.nb - tb * TILE);
        {
            const int64_t sb = P.tri0_b + min(tb * TILE + lane, P.nb - 1);
            R3<float> b0, b1, b2;
            load_tri(S.v32, S.cap, sb, b0, b1, b2);
            const PTri<float> B = prep(xform(P.Mf, P.mf, b0), xform(P.Mf, P.mf, b1), xform(P.Mf, P.mf, b2));
            float o[32];
            to_array(B, o);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                lds[lane * F32_STRIDE + q] = make_float4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
        }
        const int64_t sa = P.tri0_a + min(ia, P.na - 1);
        R3<float> a0, a1, a2;
        load_tri(S.v32, S.cap, sa, a0, a1, a2);
        const PTri<float> A = prep(a0, a1, a2);
        const int nvalid = __popcll(__ballot(a_ok));
        __syncthreads();
        const float mu = P.mu, thr2 = P.thr2, thr2_np = P.thr2_np;
        float best = big<float>(), lbA = big<float>(), lbB = big<float>();
        bool anyx = false;
        for (int j = 0; j < nbt; ++j) {
            nev += nvalid;
            float o[32];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 v = lds[j * F32_STRIDE + q];
                o[4 * q] = v.x; o[4 * q + 1] = v.y; o[4 * q + 2] = v.z; o[4 * q + 3] = v.w;
            }
            const PTri<float> B = from_array(o);
            bool np, xs;
            float d2 = pair_filter(A, B, mu, np, xs);
            d2 = a_ok ? d2 : big<float>();
            xs = xs & a_ok;
            best = fminf(best, d2);
            lbA = (!xs && !np) ? fminf(lbA, d2) : lbA;
            lbB = (!xs && np) ? fminf(lbB, d2) : lbB;
            anyx |= xs;
            const bool cand = xs | (d2 <= (np ? thr2_np : thr2));
            if (__ballot(cand)) {
                const int64_t slot = reserve(cand, cand_count);
                if (cand && slot < cand_cap)
                    cands[slot] = Cand{w.pair, (int32_t)sa, (int32_t)(P.tri0_b + tb * TILE + j), 0.f};
            }
        }
        best = wave_min(best);
        lbA = wave_min(lbA);
        lbB = wave_min(lbB);
        const bool ax = __ballot(anyx) != 0;
        if (lane == 0) {
            const float ub = sqrtf(best);
            const float lb = ax ? 0.f : fmaxf(0.f, fminf(sqrtf(lbA), sqrtf(lbB) - P.corr) - mu);
            part[it] = PartialF{ub, lb};
            atomicMin(&pair_ub[w.pair], __float_as_uint(ub + mu));
        }
        __syncthreads();
    }
    put_wave_stat(eval_slots, nev);
}

// Lexicographic (d2, i, j) minimum of two candidates.
__device__ __forceinline__ bool key_less(double d, int i, int j, double d2, int i2, int j2)
{
    return d < d2 || (d == d2 && (i < i2 || (i == i2 && j < j2)));
}

// Exact FP64 pass over every triangle pair of the items: per item the
// lexicographic minimum of (d^2, caller i, caller j); per pair the smallest
// d^2 (ties between items are settled by k_tie). With emit_cands, pairs with
// d <= delta are appended as contacts.
__global__ __launch_bounds__(64) void k_dist64(const PairDev* __restrict__ pairs, TriStore S,
                                               const Item* __restrict__ items,
                                               const int32_t* __restrict__ item_count,
                                               int64_t item_cap, PartialD* __restrict__ part,
                                               uint64_t* pair_d2, Cand* __restrict__ cands,
                                               int32_t* cand_count, int64_t cand_cap,
                                               int32_t* queue, int emit_cands,
                                               unsigned long long* eval_slots)
{
    __shared__ double2 lds[TILE * F64_STRIDE];
    __shared__ int32_t lds_orig[TILE];
    const int lane = lane_id();
    const int64_t nitems = min((int64_t)item_count[0], item_cap);
    unsigned long long nev = 0;
    int qbase = 0, qk = 4;
    for (;;) {
        const int it = pop_chunked<4>(queue, qbase, qk);
        if (it >= nitems) break;
        const Item w = items[it];
        const PairDev& P = pairs[w.pair];
        const int ta = w.tiles >> 16, tb = w.tiles & 0xffff;
        const int ia = ta * TILE + lane;
        const bool a_ok = ia < P.na;
        const int nbt = min(TILE, P.nb - tb * TILE);
        {
            const int64_t sb = P.tri0_b + min(tb * TILE + lane, P.nb - 1);
            R3<double> b0, b1, b2;
            load_tri(S.v64, S.cap, sb, b0, b1, b2);
            const PTri<double> B = prep(xform(P.M, P.m, b0), xform(P.M, P.m, b1), xform(P.M, P.m, b2));
            double o[32];
            to_array(B, o);
#pragma unroll
            for (int q = 0; q < 16; ++q) lds[lane * F64_STRIDE + q] = make_double2(o[2 * q], o[2 * q + 1]);
            lds_orig[lane] = S.orig[sb];
        }
        const int64_t sa = P.tri0_a + min(ia, P.na - 1);
        R3<double> a0, a1, a2;
        load_tri(S.v64, S.cap, sa, a0, a1, a2);
        const PTri<double> A = prep(a0, a1, a2);
        const int iorig = S.orig[sa];
        const int nvalid = __popcll(__ballot(a_ok));
        __syncthreads();
        const double dl2 = P.delta * P.delta;
        double best = 1e300;
        int bj = 0x7fffffff;
        for (int j = 0; j < nbt; ++j) {
            nev += nvalid;
            double o[32];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const double2 v = lds[j * F64_STRIDE + q];
                o[2 * q] = v.x; o[2 * q + 1] = v.y;
            }
            const PTri<double> B = from_array(o);
            int f; R3<double> xh;
            const double d2 = pair_exact<false>(A, B, f, xh);
            const int jo = lds_orig[j];
            if (a_ok && (d2 < best || (d2 == best && jo < bj))) { best = d2; bj = jo; }
            if (emit_cands) {
                const bool cand = a_ok && d2 <= dl2;
                if (__ballot(cand)) {
                    const int64_t slot = reserve(cand, cand_count);
                    if (cand && slot < cand_cap)
                        cands[slot] = Cand{w.pair, (int32_t)sa, (int32_t)(P.tri0_b + tb * TILE + j), 0.f};
                }
            }
        }
        int bi = a_ok ? iorig : 0x7fffffff;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double d2 = __shfl_xor(best, o);
            const int i2 = __shfl_xor(bi, o), j2 = __shfl_xor(bj, o);
            if (key_less(d2, i2, j2, best, bi, bj)) { best = d2; bi = i2; bj = j2; }
        }
        if (lane == 0) {
            part[it] = PartialD{best, bi, bj};
            atomicMin((unsigned long long*)&pair_d2[w.pair], (unsigned long long)__double_as_longlong(best));
        }
        __syncthreads();
    }
    put_wave_stat(eval_slots, nev);
}

// Contact-set queries in three compacted stages, so that every stage keeps
// all 64 lanes of a wave busy: the tile cull (k_cull) yields tile pairs,
// k_near tests the triangle bounding spheres of each kept tile pair and
// writes the triangle pairs whose spheres come within delta + 2 mu of each
// other to one list, and k_eval32 / k_eval64 evaluate that list one triangle
// pair per lane. Both evaluation kernels append their candidates through a
// wave-local LDS buffer that is flushed to the shared list with one atomic
// per flush.

// Plane separation of a triangle pair: B's vertices against A's plane and A's
// vertices against B's plane (planes from the FP64 vertices, FP32
// arithmetic). When all three vertices of one triangle lie more than thr =
// delta + mu beyond the other's plane on one side, the triangles are more
// than delta apart (mu covers the FP32 rounding) and cannot be in contact.
__device__ __forceinline__ bool planes_separate(const PairDev& P, R3<float> a0, R3<float> a1, R3<float> a2,
                                                R3<float> na, float oa, R3<float> b0, R3<float> b1,
                                                R3<float> b2, R3<float> nb, float ob, float thr)
{
    // B into A's frame: vertices and plane (n' = M n, off' = off + n'.m)
    const R3<float> c0 = xform(P.Mf, P.mf, b0), c1 = xform(P.Mf, P.mf, b1), c2 = xform(P.Mf, P.mf, b2);
    const R3<float> nbp = {P.Mf[0] * nb.x + P.Mf[1] * nb.y + P.Mf[2] * nb.z,
                           P.Mf[3] * nb.x + P.Mf[4] * nb.y + P.Mf[5] * nb.z,
                           P.Mf[6] * nb.x + P.Mf[7] * nb.y + P.Mf[8] * nb.z};
    const float obp = ob + dot(nbp, R3<float>{P.mf[0], P.mf[1], P.mf[2]});
    const float h0 = dot(na, c0) - oa, h1 = dot(na, c1) - oa, h2 = dot(na, c2) - oa;
    const float g0 = dot(nbp, a0) - obp, g1 = dot(nbp, a1) - obp, g2 = dot(nbp, a2) - obp;
    return (fminf(h0, fminf(h1, h2)) > thr) | (fmaxf(h0, fmaxf(h1, h2)) < -thr) |
           (fminf(g0, fminf(g1, g2)) > thr) | (fmaxf(g0, fmaxf(g1, g2)) < -thr);
}

// Triangle-sphere stage, per kept tile pair (one wave), in the order of
// growing cost:
//  1. rows: A's triangle spheres (lane = A triangle, body frame, no
//     transform) against B's tile sphere, whose centre in A's frame and
//     radius plus reach come with the item. Most kept tile pairs end here,
//     before their pair record or any B data is read;
//  2. columns: B's triangle spheres, moved into A's frame, against A's tile
//     sphere;
//  3. the remaining (row, column) pairs, packed 64 to a step, one per lane,
//     sphere against sphere.
// A pair within delta + 2 mu is written to the near list; it is marked
// "touch" when the spheres also overlap within mu (only such pairs can
// intersect). Tests counted: rows, columns and packed pairs.
constexpr int NEAR_STAGE = 512;

__global__ __launch_bounds__(64) void k_near(const PairDev* __restrict__ pairs, TriStore S,
                                             const NearItem* __restrict__ items,
                                             const int32_t* __restrict__ item_count, int64_t item_cap,
                                             int32_t* queue, NearRec* __restrict__ near,
                                             int32_t* near_count, int64_t near_cap,
                                             unsigned long long* test_slots, unsigned long long* near_slots)
{
    __shared__ float4 asph[TILE], bsph[TILE];
    __shared__ uint8_t rows[TILE], cols[TILE];
    __shared__ NearRec stage_buf[NEAR_STAGE];
    WaveStage<NearRec, NEAR_STAGE> st{stage_buf, 0};
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const int nitems = (int)min((int64_t)item_count[0], item_cap);
    unsigned long long ntest = 0, nnear = 0;
    // chunks of 16 items, fewer when the list is short for the grid (a
    // small query's few items spread over all waves instead of a few chunks)
    XcdQueue<16> wq;
    wq.init(queue, nitems, nitems / (2 * (int)gridDim.x));
    int it = wq.pop();
    if (it < 0) {
        put_wave_stat(test_slots, 0ull);
        put_wave_stat(near_slots, 0ull);
        return;
    }
    // Two-stage prefetch without branches (a finished queue repeats the last
    // valid item): the record of the item after next and the A spheres of
    // the next item are in flight while this item is processed.
    NearItem cur = items[it];
    float4 cas = S.tri_sph[cur.a0 + min(lane, cur.nat - 1)];
    int nit = wq.pop();
    NearItem nxt = items[nit >= 0 ? nit : it];
    for (;;) {
        const float4 nas = S.tri_sph[nxt.a0 + min(lane, nxt.nat - 1)];
        const int nnit = nit >= 0 ? wq.pop() : -1;
        const NearItem nnxt = items[nnit >= 0 ? nnit : (nit >= 0 ? nit : it)];
        const float4 as = cas;
        float dx = as.x - cur.cb.x, dy = as.y - cur.cb.y, dz = as.z - cur.cb.z;
        float lim = as.w + cur.cb.w;
        const uint64_t im = __ballot((lane < cur.nat) & (dx * dx + dy * dy + dz * dz <= lim * lim));
        ntest += (unsigned long long)cur.nat;
        if (im != 0) {
            const PairDev& P = pairs[cur.pair];
            const int ta = cur.tiles >> 16, tb = cur.tiles & 0xffff;
            const int nbt = min(TILE, P.nb - tb * TILE);
            const float4 braw = S.tri_sph[P.tri0_b + tb * TILE + min(lane, nbt - 1)];
            const float4 tas = S.tile_sph[P.tile0_a + ta];
            const float reach = (float)P.delta + P.mu * 2.f;
            const float mu = P.mu;
            const R3<float> cb = xform(P.Mf, P.mf, R3<float>{braw.x, braw.y, braw.z});
            const float4 bs = make_float4(cb.x, cb.y, cb.z, braw.w);
            dx = bs.x - tas.x; dy = bs.y - tas.y; dz = bs.z - tas.z;
            lim = tas.w + bs.w + reach;
            const uint64_t jm = __ballot((lane < nbt) & (dx * dx + dy * dy + dz * dz <= lim * lim));
            ntest += (unsigned long long)nbt;
            if (jm != 0) {
                // surviving rows and columns compacted: their lane and sphere
                if ((jm >> lane) & 1) {
                    const int b = __popcll(jm & below);
                    cols[b] = (uint8_t)lane;
                    bsph[b] = bs;
                }
                if ((im >> lane) & 1) {
                    const int a = __popcll(im & below);
                    rows[a] = (uint8_t)lane;
                    asph[a] = as;
                }
                __syncthreads();
                const int ni = __popcll(im), nj = __popcll(jm), np = ni * nj;
                const uint32_t pt = (uint32_t)cur.pair;
                const uint32_t ij0 = ((uint32_t)(ta * TILE) << 16) | (uint32_t)(tb * TILE);
                ntest += (unsigned long long)np;
                // q / nj through the hardware reciprocal (1 ulp): (q + 1/2) / nj
                // is at least 1/128 from an integer for q < 4096 and nj <= 64,
                // and the computed quotient is within 4096 * 2^-22 of it
                const float rnj = __builtin_amdgcn_rcpf((float)nj);
                // Plane separation of the item's staged near pairs [first, n),
                // 64 at a time, survivors compacted in place (every record of
                // a chunk is read before any is written, and writes land below
                // the chunk). The pair's transform is wave-uniform here.
                const float thr = (float)P.delta + P.mu;
                int first = st.n;
                auto plane_pass = [&]() {
                    int w = first;
                    for (int r0 = first; r0 < st.n; r0 += TILE) {
                        const int k = r0 + lane;
                        const bool has = k < st.n;
                        const NearRec rec = stage_buf[has ? k : first];
                        bool keep = false;
                        if (has) {
                            R3<float> a0, a1, a2, na, b0, b1, b2, nb;
                            float oa, ob;
                            load_tri_plane(S, P.tri0_a + (int)(rec.ij >> 16), a0, a1, a2, na, oa);
                            load_tri_plane(S, P.tri0_b + (int)(rec.ij & 0xffffu), b0, b1, b2, nb, ob);
                            keep = !planes_separate(P, a0, a1, a2, na, oa, b0, b1, b2, nb, ob, thr);
                        }
                        const uint64_t m = __ballot(keep);
                        if (keep) stage_buf[w + __popcll(m & below)] = rec;
                        w += __popcll(m);
                    }
                    nnear += (unsigned long long)(st.n - first);
                    st.n = w;
                };
                for (int q0 = 0; q0 < np; q0 += TILE) {
                    const int q = q0 + lane;
                    bool nr = false, touch = false;
                    int i = 0, j = 0;
                    if (q < np) {
                        const int a = (int)(((float)q + 0.5f) * rnj), b = q - a * nj;
                        i = rows[a];
                        j = cols[b];
                        const float4 x = asph[a], y = bsph[b];
                        const float ex = y.x - x.x, ey = y.y - x.y, ez = y.z - x.z;
                        const float g2 = ex * ex + ey * ey + ez * ez;
                        const float l = x.w + y.w + reach, lt = x.w + y.w + mu;
                        nr = g2 <= l * l;
                        touch = g2 <= lt * lt;
                    }
                    st.push(nr, NearRec{pt | (touch ? 0x80000000u : 0u), ij0 + ((uint32_t)i << 16) + (uint32_t)j});
                    if (st.n > NEAR_STAGE - TILE) {
                        plane_pass();
                        st.maybe_flush(near, near_count, near_cap);
                        first = st.n;
                    }
                }
                plane_pass();
                st.maybe_flush(near, near_count, near_cap);
                __syncthreads();
            }
        }
        if (nit < 0) break;
        it = nit;
        nit = nnit;
        cur = nxt;
        nxt = nnxt;
        cas = nas;
    }
    st.flush(near, near_count, near_cap);
    put_wave_stat(test_slots, ntest);   // ntest and nnear are wave-uniform
    put_wave_stat(near_slots, nnear);
}

// Evaluation of the near list (plane-separation survivors), one triangle pair
// per lane: the FP32 filter (candidate when its distance is within delta +
// mu, wider for near-parallel edge pairs, or when touching triangles may
// intersect) or the exact FP64 distance (candidate when d <= delta).
// Candidates go to the FP64 re-decision / closest-point pass.
template <typename T> struct EvalPass;

// Margin validation (MCD_Q_VALIDATE): the filter's distance estimate rides
// along in the candidate's float field, as d32 >= 0, or as -1 - d32 when an
// edge pair was near parallel (its bound is widened by the correction).
__device__ __forceinline__ float margin_tag(float d2, bool np) { return np ? -1.f - sqrtf(d2) : sqrtf(d2); }

template <> struct EvalPass<float> {
    static __device__ __forceinline__ bool cand(const PairDev& P, const TriStore& S, int64_t sa, int64_t sb,
                                                bool touch, bool validate, float& tag)
    {
        R3<float> a0, a1, a2, b0, b1, b2;
        load_tri_packed(S, sa, a0, a1, a2);
        load_tri_packed(S, sb, b0, b1, b2);
        const PTri<float> A = prep(a0, a1, a2);
        const PTri<float> B = prep(xform(P.Mf, P.mf, b0), xform(P.Mf, P.mf, b1), xform(P.Mf, P.mf, b2));
        bool np, xs;
        const float d2 = pair_filter(A, B, P.mu, np, xs);
        if (validate) tag = margin_tag(d2, np);
        return (xs && touch) || d2 <= (np ? P.thr2_np : P.thr2);
    }
};

template <> struct EvalPass<double> {
    static __device__ __forceinline__ bool cand(const PairDev& P, const TriStore& S, int64_t sa, int64_t sb,
                                                bool, bool, float&)
    {
        R3<double> a0, a1, a2, b0, b1, b2;
        load_tri_packed(S, sa, a0, a1, a2);
        load_tri_packed(S, sb, b0, b1, b2);
        const PTri<double> A = prep(a0, a1, a2);
        const PTri<double> B = prep(xform(P.M, P.m, b0), xform(P.M, P.m, b1), xform(P.M, P.m, b2));
        int f; R3<double> xh;
        return pair_exact<false>(A, B, f, xh) <= P.delta * P.delta;
    }
};

template <typename T>
__global__ __launch_bounds__(64) void k_eval(const PairDev* __restrict__ pairs, TriStore S,
                                             const NearRec* __restrict__ near,
                                             const int32_t* __restrict__ near_count, int64_t near_cap,
                                             Cand* __restrict__ cands, int32_t* cand_count, int64_t cand_cap,
                                             unsigned long long* eval_slots)
{
    __shared__ Cand stage_buf[CAND_STAGE];
    WaveStage<Cand, CAND_STAGE> st{stage_buf, 0};
    const int lane = lane_id();
    const int64_t n = min((int64_t)near_count[0], near_cap);
    const int64_t step = (int64_t)gridDim.x * TILE;
    int64_t base = (int64_t)blockIdx.x * TILE;
    unsigned long long nfull = 0;   // full evaluations (wave-uniform)
    NearRec rn = base < n ? near[min(base + lane, n - 1)] : NearRec{0, 0};
    for (; base < n; base += step) {
        const bool ok = base + lane < n;
        const NearRec r = rn;   // the next chunk's record is loaded one chunk ahead
        if (base + step < n) rn = near[min(base + step + lane, n - 1)];
        const int pair = (int)(r.pt & 0x7fffffffu);
        const PairDev& P = pairs[pair];
        const int64_t sa = P.tri0_a + (int)(r.ij >> 16), sb = P.tri0_b + (int)(r.ij & 0xffffu);
        // a validating query sends every evaluated pair to the FP64 re-decision
        const bool validate = ok && (P.flags & MCD_Q_VALIDATE) != 0;
        float tag = 0.f;
        const bool c = ok && EvalPass<T>::cand(P, S, sa, sb, (r.pt >> 31) != 0, validate, tag);
        nfull += (unsigned long long)min((int64_t)TILE, n - base);
        st.push(c || validate, Cand{pair, (int32_t)sa, (int32_t)sb, tag});
        st.maybe_flush(cands, cand_count, cand_cap);
    }
    st.flush(cands, cand_count, cand_cap);
    put_wave_stat(eval_slots, nfull);
}

// Items whose FP32 lower bound does not exceed their pair's FP32 upper bound
// can hold the exact minimum; they are re-run in FP64. Pairs that cannot be in
// contact are skipped unless every pair's minimum is wanted (dense).
__global__ void k_refine_select(const PairDev* __restrict__ pairs, const Item* __restrict__ items,
                                const int32_t* __restrict__ item_count, int64_t item_cap,
                                const PartialF* __restrict__ part,
                                const uint32_t* __restrict__ pair_ub, int dense,
                                Item* __restrict__ ref, int32_t* ref_count, int64_t ref_cap)
{
    const int64_t n = min((int64_t)item_count[0], item_cap);
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = base + threadIdx.x;
        bool keep = false;
        Item w{0, 0};
        if (i < n) {
            w = items[i];
            const PairDev& P = pairs[w.pair];
            float ub = __uint_as_float(pair_ub[w.pair]);
            keep = (dense || ub <= (float)P.delta + 2.f * P.mu) && part[i].lb <= ub;
        }
        int64_t slot = reserve(keep, ref_count);
        if (keep && slot < ref_cap) ref[slot] = w;
    }
}

// Ties in d^2 between items: the lowest caller (i, j) among items whose
// minimum equals the pair's minimum.
__global__ void k_tie(const Item* __restrict__ items, const int32_t* __restrict__ item_count,
                      int64_t item_cap, const PartialD* __restrict__ part,
                      const uint64_t* __restrict__ pair_d2, uint64_t* pair_tie)
{
    const int64_t n = min((int64_t)item_count[0], item_cap);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Item w = items[i];
        const PartialD q = part[i];
        if ((uint64_t)__double_as_longlong(q.d2) == pair_d2[w.pair])
            atomicMin((unsigned long long*)&pair_tie[w.pair],
                      ((unsigned long long)(uint32_t)q.ia << 32) | (uint32_t)q.jb);
    }
}

__device__ __forceinline__ void to_world(const PairDev& P, R3<double> q, double* o)
{
    R3<double> w = xform(P.Ra, P.xa, q);
    o[0] = w.x; o[1] = w.y; o[2] = w.z;
}

// FP64 re-decision of candidate triangle pairs, with closest points in the
// world frame. The squared distance comes from the same routine as the exact
// pass, so the FP64 path re-decides nothing differently.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_recheck(const PairDev* __restrict__ pairs, TriStore S,
                          const Cand* __restrict__ cands, const int32_t* __restrict__ cand_count,
                          int64_t cand_cap, CandOut* __restrict__ out, uint64_t* __restrict__ ckey,
                          uint64_t* __restrict__ cd2, uint64_t* pair_d2, int32_t* pair_cnt,
                          unsigned long long* kept_slots, unsigned long long* band_slots,
                          unsigned long long* val_slots, uint32_t* ratio_max)
{
    const int64_t n = min((int64_t)cand_count[0], cand_cap);
    unsigned long long nkept = 0, nband = 0, nval = 0;
    float rmax = 0.f, rmax_np = 0.f;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = base + threadIdx.x;
        bool keep = false, band = false, val = false;
        CandOut r;
        int rp = 0;
        double rd2 = 0.0;
        if (c < n) {
            const Cand cd = cands[c];
            const PairDev& P = pairs[cd.pair];
            R3<double> a0, a1, a2, b0, b1, b2;
            load_tri_packed(S, cd.ta, a0, a1, a2);
            load_tri_packed(S, cd.tb, b0, b1, b2);
            const PTri<double> A = prep(a0, a1, a2);
            const PTri<double> B = prep(xform(P.M, P.m, b0), xform(P.M, P.m, b1), xform(P.M, P.m, b2));
            int f; R3<double> xh;
            double d2 = pair_exact<true>(A, B, f, xh);
            keep = d2 <= P.delta * P.delta;
            // guard band: a distance this close to the threshold could be
            // decided either way by two correctly rounded FP64 evaluations
            const double dd = sqrt(d2);
            band = fabs(dd - P.delta) <= 1e-9 * P.delta;
            if ((P.flags & MCD_Q_VALIDATE) && d2 > 0.0) {
                const float tg = cd.t;
                const bool np = tg < 0.f;
                const double d32 = np ? -1.0 - (double)tg : (double)tg;
                if (np) rmax_np = fmaxf(rmax_np, (float)(fabs(d32 - dd) / ((double)P.mu + (double)P.corr)));
                else rmax = fmaxf(rmax, (float)(fabs(d32 - dd) / (double)P.mu));
                val = true;
            }
            if (keep) {
                R3<double> qa, qb;
                feature_points(A, B, f, xh, qa, qb);
                r.d = sqrt(d2);
                to_world(P, qa, r.pa);
                to_world(P, qb, r.pb);
                r.pair = cd.pair;
                r.tri_a = S.orig[cd.ta];
                r.tri_b = S.orig[cd.tb];
                r.keep = 1;
                r.d2 = d2;
                rp = cd.pair;
                rd2 = d2;
            }
            // one record per candidate, at its own index (no shared counter),
            // and its (pair, tri_a, tri_b) key for the per-pair ordering
            if (keep) out[c] = r;
            else out[c].keep = 0;
            ckey[c] = keep ? ((uint64_t)(uint32_t)cd.pair << 32) | ((uint64_t)(uint32_t)r.tri_a << 16) |
                                 (uint32_t)r.tri_b
                           : ~0ull;
            cd2[c] = keep ? (uint64_t)__double_as_longlong(rd2) : ~0ull;
        }
        // a pair in contact has its minimum among its contacts
        wave_min_by_key(keep, rp, (uint64_t)__double_as_longlong(rd2), pair_d2);
        wave_count_by_key(keep, rp, pair_cnt);
        nkept += __popcll(__ballot(keep));
        nband += __popcll(__ballot(band));
        nval += __popcll(__ballot(val));
    }
    put_wave_stat(kept_slots, nkept);
    put_wave_stat(band_slots, nband);
    put_wave_stat(val_slots, nval);
    // largest ratios of the wave (validating queries only): one atomic each
    // per wave; ratio_max[0] pairs without, ratio_max[1] pairs with a
    // near-parallel edge pair
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmaxf(rmax, __shfl_xor(rmax, o));
        rmax_np = fmaxf(rmax_np, __shfl_xor(rmax_np, o));
    }
    if (nval > 0 && lane_id() == 0) {
        atomicMax(&ratio_max[0], __float_as_uint(rmax));
        atomicMax(&ratio_max[1], __float_as_uint(rmax_np));
    }
}

// Per pair: closest points of the winning triangle pair. Reported when the
// pair is in contact (d <= delta), or always when the query is dense.
__device__ __forceinline__ void pair_final_one(const PairDev* __restrict__ pairs, int p, const TriStore& S,
                                               const uint64_t* __restrict__ pair_d2,
                                               const uint64_t* __restrict__ pair_tie, int dense,
                                               PairOut* __restrict__ out)
{
    const PairDev& P = pairs[p];
    PairOut r;
    r.toi = 0.0;
    r.status = 0;
    const uint64_t k = pair_d2[p];
    const uint64_t t = pair_tie[p];
    double d2 = __longlong_as_double((long long)k);
    bool have = k != ~0ull && t != ~0ull && d2 < 1e299;
    bool contact = have && d2 <= P.delta * P.delta;
    if (!have || !(contact || dense)) {
        r.d = __longlong_as_double(0x7ff0000000000000ll);
        r.pa[0] = r.pa[1] = r.pa[2] = r.pb[0] = r.pb[1] = r.pb[2] = 0.0;
        r.tri_a = r.tri_b = -1;
        r.contact = 0;
        out[p] = r;
        return;
    }
    const int io = (int)(t >> 32), jo = (int)(t & 0xffffffffu);
    const int64_t sa = S.pos[P.tri0_a + io], sb = S.pos[P.tri0_b + jo];
    R3<double> a0, a1, a2, b0, b1, b2;
    load_tri_packed(S, sa, a0, a1, a2);
    load_tri_packed(S, sb, b0, b1, b2);
    const PTri<double> A = prep(a0, a1, a2);
    const PTri<double> B = prep(xform(P.M, P.m, b0), xform(P.M, P.m, b1), xform(P.M, P.m, b2));
    int f; R3<double> xh, qa, qb;
    double e2 = pair_exact<true>(A, B, f, xh);
    feature_points(A, B, f, xh, qa, qb);
    r.d = sqrt(e2);
    to_world(P, qa, r.pa);
    to_world(P, qb, r.pb);
    r.tri_a = io;
    r.tri_b = jo;
    r.contact = contact ? 1 : 0;
    r.status = r.contact;
    out[p] = r;
}

__global__ __launch_bounds__(64) void k_pair_final(const PairDev* __restrict__ pairs, const int32_t* nq,
                             int32_t ncap, TriStore S, const uint64_t* __restrict__ pair_d2,
                             const uint64_t* __restrict__ pair_tie, int dense,
                             PairOut* __restrict__ out)
{
    const int npairs = min(nq[0], ncap);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npairs; p += gridDim.x * blockDim.x)
        pair_final_one(pairs, p, S, pair_d2, pair_tie, dense, out);
}

// Ties between contacts of equal minimal d^2: the lowest caller (i, j).
__global__ void k_tie_out(const uint64_t* __restrict__ ckey, const uint64_t* __restrict__ cd2,
                          const int32_t* __restrict__ count, int64_t cap,
                          const uint64_t* __restrict__ pair_d2, uint64_t* pair_tie)
{
    const int64_t n = min((int64_t)count[0], cap);
    // the loop runs wave-uniformly: lanes past the end take part without a
    // record, so that the per-wave combination below sees the whole wave
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = b + threadIdx.x;
        const uint64_t k = i < n ? ckey[i] : ~0ull;
        const int p = (int)(k >> 32);
        const bool at_min = k != ~0ull && cd2[i] == pair_d2[p];
        // contacts of one pair sit mostly in one wave (touching triangles at
        // d = 0 share the minimum): one atomic per distinct pair of the wave
        wave_min_by_key(at_min, p, ((uint64_t)((k >> 16) & 0xffffu) << 32) | (uint32_t)(k & 0xffffu), pair_tie);
    }
}

// Exclusive scan of the per-pair contact counts and the largest count (one
// block of 1024 threads; each thread a run of 8 consecutive pairs per pass).
__global__ __launch_bounds__(1024) void k_pair_scan(const int32_t* __restrict__ nq,
                                                    const int32_t* __restrict__ cnt, int32_t* off,
                                                    int32_t* max_seg, int32_t* __restrict__ large)
{
    __shared__ int32_t wsum[16], wmax[16];
    __shared__ int32_t nlarge;
    const int n = nq[0], t = threadIdx.x, lane = lane_id(), w = t / 64;
    if (t == 0) nlarge = 0;
    __syncthreads();
    constexpr int RUN = 8;
    int carry = 0, mx = 0;
    for (int base = 0; base < n; base += 1024 * RUN) {
        const int lo = base + t * RUN;
        int v[RUN], sum = 0, m = 0;
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            v[k] = lo + k < n ? cnt[lo + k] : 0;
            sum += v[k];
            m = max(m, v[k]);
        }
        int x = sum;   // inclusive scan of the run totals within the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
        if (lane == 63) wsum[w] = x;
        if (lane == 0) wmax[w] = m;
        __syncthreads();
        int before = 0, total = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) before += wsum[k];
            total += wsum[k];
            mx = max(mx, wmax[k]);
        }
        int run = carry + before + x - sum;
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            if (lo + k < n) off[lo + k] = run;
            if (v[k] > 64) large[atomicAdd(&nlarge, 1)] = lo + k;   // pairs for the LDS sort
            run += v[k];
        }
        carry += total;
        __syncthreads();
    }
    __syncthreads();
    if (t == 0) {
        off[n] = carry;
        max_seg[0] = mx;
        max_seg[1] = nlarge;
    }
}

// Each contact to a slot of its pair's segment: per distinct pair of the wave
// one atomic on the pair's remaining count.
__global__ void k_contact_scatter(const uint64_t* __restrict__ ckey, int32_t n, const int32_t* __restrict__ off,
                                  int32_t* cursor, uint64_t* __restrict__ seg)
{
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t i = base + lane;
        bool keep = false;
        int p = 0;
        uint32_t tt = 0;
        if (i < n) {
            const uint64_t k = ckey[i];
            keep = k != ~0ull;
            p = (int)(k >> 32);
            tt = (uint32_t)k;
        }
        uint64_t pending = __ballot(keep);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int k = __builtin_amdgcn_readlane(p, leader);
            const uint64_t same = __ballot(keep && p == k);
            int top = 0;
            if (lane == leader) top = atomicSub(&cursor[k], (int)__popcll(same));
            top = __shfl(top, leader);
            if (keep && p == k)
                seg[off[k] + top - 1 - __popcll(same & below)] = ((uint64_t)tt << 32) | (uint32_t)i;
            pending &= ~same;
        }
    }
}

__device__ __forceinline__ void put_contact(const CandOut& o, mcd_contact* dst)
{
    mcd_contact c;
    c.pair = o.pair; c.tri_a = o.tri_a; c.tri_b = o.tri_b; c.merged = 0;
    c.d = o.d;
    c.pa[0] = o.pa[0]; c.pa[1] = o.pa[1]; c.pa[2] = o.pa[2];
    c.pb[0] = o.pb[0]; c.pb[1] = o.pb[1]; c.pb[2] = o.pb[2];
    c.t = 0.0;   // the runtime sets the pair's time stamp for time queries
    *dst = c;
}

// One wave per pair with at most 64 contacts: its segment (keys (tri_a,
// tri_b) above the record index) sorted by a bitonic network through lane
// exchanges, then the contact records written in that order.
__global__ __launch_bounds__(64) void k_segment_sort_small(const CandOut* __restrict__ out,
                                                           const int32_t* __restrict__ off,
                                                           const uint64_t* __restrict__ seg,
                                                           mcd_contact* __restrict__ dst)
{
    const int p = blockIdx.x, lane = lane_id();
    const int o0 = off[p], m = off[p + 1] - o0;
    if (m <= 0 || m > 64) return;
    unsigned long long x = lane < m ? seg[o0 + lane] : ~0ull;
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned long long y = __shfl_xor(x, j);
            const bool up = (lane & k) == 0, low = (lane & j) == 0;
            x = (low == up) ? (x < y ? x : y) : (x < y ? y : x);
        }
    }
    if (lane < m) put_contact(out[(uint32_t)x], dst + o0 + lane);
}

// One block per pair with 65 to SEG_CAP contacts (the list `large` from the
// pair scan; 256 to 1024 threads, half the largest segment's power of two):
// the same bitonic network over a power-of-two array (p2 <= 4 x blockDim
// keys). Key i sits in lane i % 64 of its wave, so every compare-exchange
// at a distance below 64 is a shuffle within the wave on keys held in
// registers (the first 21 steps at once, then the last 6 of each merge).
// Only the steps at distance 64 and more go through LDS, one pair per
// thread, each followed by a barrier.
constexpr int SORT_KEYS_PER_THREAD = SEG_CAP / 1024;

__device__ __forceinline__ void bitonic_regs(uint64_t (&x)[SORT_KEYS_PER_THREAD], int t, int nt, int p2, int k0,
                                             int k1, int j0)
{
    for (int k = k0; k <= k1; k <<= 1) {
        for (int j = (k == k0 ? j0 : k >> 1); j > 0; j >>= 1) {
#pragma unroll
            for (int r = 0; r < SORT_KEYS_PER_THREAD; ++r) {
                if (r * nt < p2) {   // block-uniform
                    const int i = t + r * nt;
                    const uint64_t y = __shfl_xor(x[r], j);
                    const bool up = (i & k) == 0, low = (i & j) == 0;
                    x[r] = (low == up) ? (x[r] < y ? x[r] : y) : (x[r] < y ? y : x[r]);
                }
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_segment_sort_large(const CandOut* __restrict__ out,
                                                             const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ large,
                                                             const uint64_t* __restrict__ seg, int p2max,
                                                             mcd_contact* __restrict__ dst)
{
    extern __shared__ uint64_t a[];
    const int p = large[blockIdx.x], t = threadIdx.x, nt = blockDim.x;
    const int o0 = off[p], m = off[p + 1] - o0;
    if (m <= 64) return;
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    if (p2 > p2max || p2 > SORT_KEYS_PER_THREAD * nt) return;   // the host sized both for the largest segment
    uint64_t x[SORT_KEYS_PER_THREAD];
#pragma unroll
    for (int r = 0; r < SORT_KEYS_PER_THREAD; ++r) {
        const int i = t + r * nt;
        x[r] = i < m ? seg[o0 + i] : ~0ull;
    }
    // merges of width 2 to 64: within the wave
    bitonic_regs(x, t, nt, p2, 2, 64, 1);
    for (int k = 128; k <= p2; k <<= 1) {
#pragma unroll
        for (int r = 0; r < SORT_KEYS_PER_THREAD; ++r)
            if (t + r * nt < p2) a[t + r * nt] = x[r];
        __syncthreads();
        for (int j = k >> 1; j >= 64; j >>= 1) {
            for (int q = t; q < (p2 >> 1); q += nt) {
                const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1)), l = i | j;
                const uint64_t u = a[i], v = a[l];
                if ((u > v) == ((i & k) == 0)) { a[i] = v; a[l] = u; }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < SORT_KEYS_PER_THREAD; ++r)
            if (t + r * nt < p2) x[r] = a[t + r * nt];
        __syncthreads();   // every key read back before the next merge stores
        bitonic_regs(x, t, nt, p2, k, k, 32);
    }
#pragma unroll
    for (int r = 0; r < SORT_KEYS_PER_THREAD; ++r) {
        const int i = t + r * nt;
        if (i < m) put_contact(out[(uint32_t)x[r]], dst + o0 + i);
    }
}

__global__ void k_contact_keys(const CandOut* __restrict__ out, int32_t n, int tri_bits, uint64_t none,
                               uint64_t* __restrict__ keys, int32_t* __restrict__ idx)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const CandOut& o = out[i];
        // (pair, tri_a, tri_b) packed in as few bits as the query needs;
        // records without a contact sort after every contact
        keys[i] = o.keep ? ((((uint64_t)(uint32_t)o.pair << tri_bits) | (uint32_t)o.tri_a) << tri_bits) | (uint32_t)o.tri_b
                         : none;
        idx[i] = i;
    }
}

__global__ void k_contact_gather(const CandOut* __restrict__ out, int32_t n, const int32_t* __restrict__ idx,
                                 mcd_contact* __restrict__ dst)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        put_contact(out[idx[i]], dst + i);
    }
}

inline int grid_for(int64_t n, int block, int cap_blocks)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_u64(const Launch& L, uint64_t* p, int64_t n, uint64_t v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, L.stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(const Launch& L, uint32_t* p, int64_t n, uint32_t v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, L.stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_pair_prep(const Launch& L, const int32_t* hdr_src, const PairSrc* src, int32_t ncap,
                            const PrepOpts& o, int32_t* hdr_dst, PairDev* out, const uint64_t* tkey,
                            const double* tval, int tmode)
{
    hipLaunchKernelGGL(k_pair_prep, dim3(grid_for(ncap > 0 ? ncap : 1, 128, 1024)), dim3(128), 0, L.stream,
                       hdr_src, src, ncap, o, hdr_dst, out, tkey, tval, tmode);
    return hipGetLastError();
}

hipError_t launch_pair_gather(const Launch& L, const int32_t* nlist, const int32_t* dlist, int32_t ncap,
                              const PartDev* parts, int32_t npart, const MeshDev* meshes, int32_t nmesh,
                              double t, int toi, int32_t rows, int64_t item_cap, int64_t word_cap,
                              int32_t* hdr_src, PairSrc* src, int64_t* tmp, int32_t* counters, int err_word,
                              int words_at, int tiles_at, int tris_at)
{
    hipLaunchKernelGGL(k_pair_gather, dim3(grid_for(ncap > 0 ? ncap : 1, 256, 1 << 16)), dim3(256), 0, L.stream,
                       nlist, dlist, ncap, parts, npart, meshes, nmesh, t, toi, rows, hdr_src, src, tmp, counters,
                       err_word);
    hipLaunchKernelGGL(k_pair_offsets, dim3(1), dim3(1024), 0, L.stream, nlist, ncap, toi, item_cap, word_cap, src,
                       tmp, counters, err_word, words_at, tiles_at, tris_at);
    return hipGetLastError();
}

hipError_t launch_part_scatter(const Launch& L, const int32_t* ids, const PartDev* recs, int32_t n,
                               PartDev* table)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_part_scatter, dim3(grid_for(n, 256, 1024)), dim3(256), 0, L.stream, ids, recs, n, table);
    return hipGetLastError();
}

hipError_t launch_init_static(const Launch& L, uint32_t* counters, int ncounters, uint32_t* pair_ub,
                              uint64_t* pair_d2, uint64_t* pair_tie, int32_t* pair_cnt, int32_t ncap)
{
    const int n = ncap > ncounters ? ncap : ncounters;
    hipLaunchKernelGGL(k_init_static, dim3(grid_for(n, 256, 1024)), dim3(256), 0, L.stream, counters,
                       ncounters, pair_ub, pair_d2, pair_tie, pair_cnt, ncap);
    return hipGetLastError();
}

int cull_grid(const Launch& L, int32_t ncap) { return ncap < L.num_cu * 32 ? (ncap > 0 ? ncap : 1) : L.num_cu * 32; }

hipError_t launch_cull(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t ncap, const TriStore& S,
                       int dense, Item* items, NearItem* near_items, int32_t* item_count, int64_t item_cap,
                       unsigned long long* tiled_count, int32_t* scan_buf, uint64_t* mask,
                       unsigned long long* test_slots)
{
    if (ncap <= 0) return hipSuccess;
    int32_t* pcount = scan_buf;
    int32_t* poff = scan_buf + ncap;
    int64_t* ptiled = (int64_t*)(scan_buf + 2 * ((ncap + 1) & ~1));
    const int grid = cull_grid(L, ncap);
    hipLaunchKernelGGL(k_cull_count, dim3(grid), dim3(256), 0, L.stream, pairs, nq, ncap, S, dense, pcount,
                       ptiled, mask, test_slots);
    hipLaunchKernelGGL(k_cull_scan, dim3(1), dim3(1024), 0, L.stream, pcount, ptiled, nq, ncap, poff,
                       item_count, tiled_count);
    hipLaunchKernelGGL(k_cull_write, dim3(grid), dim3(256), 0, L.stream, pairs, nq, ncap, S, poff, mask,
                       dense, items, near_items, item_cap);
    return hipGetLastError();
}

hipError_t launch_dist32(const Launch& L, const PairDev* pairs, const TriStore& S,
                         const Item* items, const int32_t* item_count, int64_t item_cap,
                         PartialF* part, uint32_t* pair_ub, Cand* cands, int32_t* cand_count,
                         int64_t cand_cap, int32_t* queue, unsigned long long* eval_slots, int grid)
{
    hipLaunchKernelGGL(k_dist32, dim3(grid), dim3(64), 0, L.stream, pairs, S, items, item_count, item_cap,
                       part, pair_ub, cands, cand_count, cand_cap, queue, eval_slots);
    return hipGetLastError();
}

hipError_t launch_dist64(const Launch& L, const PairDev* pairs, const TriStore& S,
                         const Item* items, const int32_t* item_count, int64_t item_cap,
                         PartialD* part, uint64_t* pair_d2, Cand* cands, int32_t* cand_count,
                         int64_t cand_cap, int32_t* queue, int emit_cands,
                         unsigned long long* eval_slots, int grid)
{
    hipLaunchKernelGGL(k_dist64, dim3(grid), dim3(64), 0, L.stream, pairs, S, items, item_count, item_cap,
                       part, pair_d2, cands, cand_count, cand_cap, queue, emit_cands, eval_slots);
    return hipGetLastError();
}

hipError_t launch_near(const Launch& L, const PairDev* pairs, const TriStore& S, const NearItem* items,
                       const int32_t* item_count, int64_t item_cap, int32_t* queue, NearRec* near,
                       int32_t* near_count, int64_t near_cap, unsigned long long* test_slots,
                       unsigned long long* near_slots, int grid)
{
    hipLaunchKernelGGL(k_near, dim3(grid * 2), dim3(64), 0, L.stream, pairs, S, items, item_count, item_cap,
                       queue, near, near_count, near_cap, test_slots, near_slots);
    return hipGetLastError();
}

hipError_t launch_eval(const Launch& L, bool fp64, const PairDev* pairs, const TriStore& S,
                       const NearRec* near, const int32_t* near_count, int64_t near_cap, Cand* cands,
                       int32_t* cand_count, int64_t cand_cap, unsigned long long* eval_slots, int grid)
{
    if (fp64)
        hipLaunchKernelGGL(k_eval<double>, dim3(grid), dim3(64), 0, L.stream, pairs, S, near, near_count,
                           near_cap, cands, cand_count, cand_cap, eval_slots);
    else
        hipLaunchKernelGGL(k_eval<float>, dim3(grid), dim3(64), 0, L.stream, pairs, S, near, near_count,
                           near_cap, cands, cand_count, cand_cap, eval_slots);
    return hipGetLastError();
}

hipError_t launch_refine_select(const Launch& L, const PairDev* pairs, const Item* items,
                                const int32_t* item_count, int64_t item_cap, const PartialF* part,
                                const uint32_t* pair_ub, int dense, Item* ref_items,
                                int32_t* ref_count, int64_t ref_cap)
{
    hipLaunchKernelGGL(k_refine_select, dim3(grid_for(item_cap, 256, 2048)), dim3(256), 0,
                       L.stream, pairs, items, item_count, item_cap, part, pair_ub, dense,
                       ref_items, ref_count, ref_cap);
    return hipGetLastError();
}

hipError_t launch_tie(const Launch& L, const Item* items, const int32_t* item_count,
                      int64_t item_cap, const PartialD* part, const uint64_t* pair_d2,
                      uint64_t* pair_tie)
{
    hipLaunchKernelGGL(k_tie, dim3(grid_for(item_cap, 256, 2048)), dim3(256), 0, L.stream, items,
                       item_count, item_cap, part, pair_d2, pair_tie);
    return hipGetLastError();
}

int recheck_grid(int64_t cand_cap) { return grid_for(cand_cap, 64, 8192); }

hipError_t launch_recheck(const Launch& L, const PairDev* pairs, const TriStore& S,
                          const Cand* cands, const int32_t* cand_count, int64_t cand_cap,
                          CandOut* out, uint64_t* ckey, uint64_t* cd2, uint64_t* pair_d2, int32_t* pair_cnt,
                          unsigned long long* kept_slots, unsigned long long* band_slots,
                          unsigned long long* val_slots, uint32_t* ratio_max)
{
    hipLaunchKernelGGL(k_recheck, dim3(recheck_grid(cand_cap)), dim3(64), 0, L.stream,
                       pairs, S, cands, cand_count, cand_cap, out, ckey, cd2, pair_d2, pair_cnt, kept_slots,
                       band_slots, val_slots, ratio_max);
    return hipGetLastError();
}

hipError_t launch_pair_final(const Launch& L, const PairDev* pairs, const int32_t* nq, int32_t ncap,
                             const TriStore& S, const uint64_t* pair_d2, const uint64_t* pair_tie,
                             int dense, PairOut* out)
{
    if (ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_final, dim3(grid_for(ncap, 64, 4096)), dim3(64), 0, L.stream, pairs,
                       nq, ncap, S, pair_d2, pair_tie, dense, out);
    return hipGetLastError();
}

hipError_t launch_stat_reduce(const Launch& L, const uint64_t* slots, const StatPlan& plan,
                              unsigned long long* counters64)
{
    if (plan.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stat_reduce, dim3(plan.n * STAT_PARTS), dim3(256), 0, L.stream, slots, plan, counters64);
    return hipGetLastError();
}

hipError_t launch_tie_out(const Launch& L, const uint64_t* ckey, const uint64_t* cd2, const int32_t* count,
                          int64_t cap, const uint64_t* pair_d2, uint64_t* pair_tie)
{
    hipLaunchKernelGGL(k_tie_out, dim3(grid_for(cap, 256, 2048)), dim3(256), 0, L.stream, ckey, cd2,
                       count, cap, pair_d2, pair_tie);
    return hipGetLastError();
}

hipError_t launch_pair_scan(const Launch& L, const int32_t* nq, const int32_t* pair_cnt, int32_t* pair_off,
                            int32_t* max_seg, int32_t* large)
{
    hipLaunchKernelGGL(k_pair_scan, dim3(1), dim3(1024), 0, L.stream, nq, pair_cnt, pair_off, max_seg, large);
    return hipGetLastError();
}

hipError_t sort_contacts_by_pair(const Launch& L, const CandOut* out, const uint64_t* ckey, int32_t n,
                                 int32_t npairs, const int32_t* pair_off, int32_t* pair_cnt,
                                 const int32_t* large, int32_t nlarge, uint64_t* seg, int seg_p2,
                                 mcd_contact* sorted)
{
    if (n <= 0 || npairs <= 0) return hipSuccess;
    if (seg_p2 < 1 || seg_p2 > SEG_CAP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_contact_scatter, dim3(grid_for(n, 256, 4096)), dim3(256), 0, L.stream, ckey, n,
                       pair_off, pair_cnt, seg);
    hipLaunchKernelGGL(k_segment_sort_small, dim3(npairs), dim3(64), 0, L.stream, out, pair_off, seg, sorted);
    if (seg_p2 > 64 && nlarge > 0) {
        const int threads = seg_p2 / 2 < 256 ? 256 : (seg_p2 / 2 > 1024 ? 1024 : seg_p2 / 2);
        hipLaunchKernelGGL(k_segment_sort_large, dim3(nlarge), dim3(threads), sizeof(uint64_t) * seg_p2, L.stream,
                           out, pair_off, large, seg, seg_p2, sorted);
    }
    return hipGetLastError();
}

hipError_t sort_contacts(const Launch& L, const CandOut* out, int32_t n, int32_t ncon, int pair_bits,
                         int tri_bits, uint64_t* keys, uint64_t* keys_alt, int32_t* idx, int32_t* idx_alt,
                         void* temp, size_t& temp_bytes, mcd_contact* sorted)
{
    // key bits: pair, tri_a, tri_b, and one above them for records without contact
    const int bits = pair_bits + 2 * tri_bits;
    if (bits + 1 > 64) return hipErrorInvalidValue;
    // rocprim picks a merge sort below a million keys (nine merge passes here);
    // a limit of 0 keeps the onesweep radix sort, ceil((bits + 1) / 8) passes.
    using OnesweepOnly = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                    rocprim::default_config, 0>;
    if (!temp)
        return rocprim::radix_sort_pairs<OnesweepOnly>(nullptr, temp_bytes, keys, keys_alt, idx, idx_alt,
                                                       n > 0 ? n : 1, 0, bits + 1, L.stream);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_contact_keys, dim3(grid_for(n, 256, 4096)), dim3(256), 0, L.stream, out, n,
                       tri_bits, (uint64_t)1 << bits, keys, idx);
    hipError_t e = rocprim::radix_sort_pairs<OnesweepOnly>(temp, temp_bytes, keys, keys_alt, idx, idx_alt,
                                                           n, 0, bits + 1, L.stream);
    if (e != hipSuccess) return e;
    if (ncon <= 0) return hipGetLastError();
    hipLaunchKernelGGL(k_contact_gather, dim3(grid_for(ncon, 256, 4096)), dim3(256), 0, L.stream, out, ncon,
                       idx_alt, sorted);
    return hipGetLastError();
}

}  // namespace mcd
