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
// GPU split: (1) a space-time tile cull moves the tile bounding spheres to
// every sample time and keeps a tile pair only if some interval cannot be
// excluded, recording the first such interval and a distance bound; (2) the
// sampler works on compacted lists so that every lane of a wave has work:
// per kept tile pair, the triangles' bounding spheres take the first steps of
// a Lipschitz walk through the sample times (stage 1); walks still undecided
// continue one per lane, idle lanes refilled from the list (stage 1b); pairs
// whose spheres come within the threshold walk their triangles in FP32 with
// margin mu, again one per lane with refill (stage 2), and hand the first
// interval they cannot clear to (3) an FP64 end-game that runs the exact
// interval logic (sampling, halving, bisection) from there on, 16 lanes per
// candidate. Intervals cleared before hold no time with d <= delta, so the
// end-game returns the same time as the plain scan over every interval. Per
// pair the earliest (time, i, j) wins through one 64-bit atomic minimum on
// lattice keys.
#include "mcd_internal.h"
#include "mcd_geom.h"
#include "mcd_dev.h"

namespace mcd {

namespace {

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

// Relative transforms at the S+1 sample times of every pair (FP32 and FP64
// copies, 12 values per row: M row-major, then m).
__global__ void k_toi_table(const PairDev* __restrict__ pairs, int32_t npairs, int32_t rows,
                            float* __restrict__ table32, double* __restrict__ table64)
{
    const int64_t n = (int64_t)npairs * rows;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / rows), k = (int)(i - (int64_t)p * rows);
        const PairDev& P = pairs[p];
        if (k > P.samples) continue;
        double M[9], m[3];
        rel_at(P, sample_time(k, P.dt, P.samples), M, m);
        float* o = table32 + (P.table0 + k) * 12;
        double* o64 = table64 + (P.table0 + k) * 12;
#pragma unroll
        for (int j = 0; j < 9; ++j) { o[j] = (float)M[j]; o64[j] = M[j]; }
#pragma unroll
        for (int j = 0; j < 3; ++j) { o[9 + j] = (float)m[j]; o64[9 + j] = m[j]; }
    }
}

// Space-time tile cull. The distance between any triangles of two tiles is at
// least D(t) = |c_a - c_b(t)| - r_a - r_b (bounding spheres), and D changes at
// most at rate Lc = |v_a - v_b| + |w_a| |c_a| + |w_b| |c_b| (sphere centres
// about the rotation centres). A tile pair is kept from the first sample
// interval whose end values or envelope (D_k + D_k+1 - Lc h)/2 come within
// delta + mu; earlier intervals are contact-free for all its triangle pairs.
constexpr int MAX_ROWS = 129;   // samples S <= 128
constexpr int MAX_GROUP_PAIRS = 1024;   // group pairs a block holds (larger pairs skip the group level)

// The first sample interval from k0 on that two spheres (a, b: centres in
// their body frames, radii) cannot be shown apart over, or -1: end values or
// envelope (D_k + D_k+1 - Lc h)/2 within thr. dlb receives the lower bound
// at that interval's start.
__device__ __forceinline__ int sphere_first(const float* tab, int Sn, int k0, float4 a, float4 b, float Lc, float h,
                                            float thr, float& dlb)
{
    const float rr = a.w + b.w;
    float dprev = 0.f;
    for (int k = k0; k <= Sn; ++k) {
        const float* T = tab + 12 * k;
        const R3<float> c = xform(T, T + 9, R3<float>{b.x, b.y, b.z});
        const float dx = c.x - a.x, dy = c.y - a.y, dz = c.z - a.z;
        const float dn = fsqrt(dx * dx + dy * dy + dz * dz) - rr;
        if (k == k0) {
            if (k == 0 && dn <= thr) { dlb = dn; return 0; }
        } else if (dn <= thr || (dprev + dn - Lc * h) * 0.5f <= thr) {
            dlb = dprev;
            return k - 1;
        }
        dprev = dn;
    }
    return -1;
}

__global__ __launch_bounds__(256) void k_toi_cull(const PairDev* __restrict__ pairs, TriStore S,
                                                  const float* __restrict__ table,
                                                  ToiItem* __restrict__ items)
{
    __shared__ float tab[MAX_ROWS * 12];
    __shared__ int16_t gfirst[MAX_GROUP_PAIRS];
    const int p = blockIdx.x;
    const PairDev& P = pairs[p];
    const int Sn = P.samples;
    for (int i = threadIdx.x; i < (Sn + 1) * 12; i += blockDim.x) tab[i] = table[P.table0 * 12 + i];
    __syncthreads();
    const float h = (float)(P.dt / Sn);
    const float slack = 1e-6f * (float)(P.L * P.dt);
    const float thr = (float)P.delta + P.mu + slack;
    const int nta = P.nta, ntb = P.ntb, ntot = nta * ntb;
    // Group level: each group pair's first interval its spheres cannot
    // exclude (-1: none); its tile pairs start there. Intervals excluded for
    // the group spheres are contact-free for every triangle pair under them.
    const int nga = (nta + GROUP - 1) / GROUP, ngb = (ntb + GROUP - 1) / GROUP;
    const bool grouped = nga * ngb <= MAX_GROUP_PAIRS && nga * ngb > 1;
    if (grouped) {
        for (int g = threadIdx.x; g < nga * ngb; g += blockDim.x) {
            const int ga = g / ngb, gb = g - ga * ngb;
            const float4 a = S.grp_sph[P.group0_a + ga];
            const float4 b = S.grp_sph[P.group0_b + gb];
            const float ra = fsqrt(a.x * a.x + a.y * a.y + a.z * a.z);
            const float rb = fsqrt(b.x * b.x + b.y * b.y + b.z * b.z);
            const float Lc = (P.vr + P.wa * ra + P.wb * rb) * (1.f + 1e-6f);
            float dlb;
            gfirst[g] = (int16_t)sphere_first(tab, Sn, 0, a, b, Lc, h, thr + P.mu, dlb);
        }
        __syncthreads();
    }
    for (int base = 0; base < ntot; base += blockDim.x) {
        const int q = base + threadIdx.x;
        bool keep = false;
        int ta = 0, tb = 0, kf = 0;
        float dlb = 0.f;
        if (q < ntot) {
            ta = q / ntb;
            tb = q - ta * ntb;
            const int k0 = grouped ? gfirst[(ta / GROUP) * ngb + tb / GROUP] : 0;
            if (k0 >= 0) {
                const float4 a = S.tile_sph[P.tile0_a + ta];
                const float4 b = S.tile_sph[P.tile0_b + tb];
                const float ra = fsqrt(a.x * a.x + a.y * a.y + a.z * a.z);
                const float rb = fsqrt(b.x * b.x + b.y * b.y + b.z * b.z);
                const float Lc = (P.vr + P.wa * ra + P.wb * rb) * (1.f + 1e-6f);
                kf = sphere_first(tab, Sn, k0, a, b, Lc, h, thr, dlb);
                keep = kf >= 0;
            }
        }
        // every tile pair has its slot: no shared counter to wait on
        if (q < ntot) items[P.tp0 + q] = ToiItem{p, (ta << 16) | tb, keep ? kf : -1, dlb};
    }
}

// One sample: B's triangle (body frame) moved by row T, prepared, measured
// against A. dlb: lower bound of the true distance; dub: the feature distance
// (an upper bound within mu); xs: the two triangles may intersect.
__device__ __forceinline__ void sample_eval(const PTri<float>& A, const float* T, R3<float> b0,
                                            R3<float> b1, R3<float> b2, float mu, float corr,
                                            float& dlb, float& dub, bool& xs)
{
    const PTri<float> B = prep(xform(T, T + 9, b0), xform(T, T + 9, b1), xform(T, T + 9, b2));
    bool np;
    const float d2 = pair_filter(A, B, mu, np, xs);
    dub = fsqrt(d2);
    dlb = xs ? 0.f : fmaxf(0.f, dub - (np ? corr : 0.f));
}

__device__ __forceinline__ void sample_eval(const PTri<double>& A, const double* T, R3<double> b0,
                                            R3<double> b1, R3<double> b2, double mu, double corr,
                                            double& dlb, double& dub, bool& xs)
{
    const PTri<double> B = prep(xform(T, T + 9, b0), xform(T, T + 9, b1), xform(T, T + 9, b2));
    int f;
    R3<double> x;
    dub = sqrt(pair_exact<false>(A, B, f, x));
    dlb = fmax(0.0, dub - corr);
    xs = false;
    (void)mu;
}

// Bounding-sphere walk through the sample times. From a point (ts, ds) with
// ds a lower bound of every triangle distance the two spheres cover, the
// gap of the two spheres changes no faster than Ls = |v_a - v_b| + |w_a| |c_a|
// + |w_b| |c_b| (their centres about the rotation centres; at most the pair's
// L), which proves d > delta + margins until need = ts + (ds - thr)/Ls;
// the sphere gap (less mu) at the last sample before need is the next lower
// bound. A walk ends when the spheres clear the step or pass the pair's
// proven-contact sample (SW_CLEAR), or when the gap falls within the
// threshold (SW_NEAR; (ke, ds) is then the last proven point: ke = -1 means
// ds bounds the distance at the start sample kf). SW_MORE: the step budget
// ran out first.
enum { SW_CLEAR = 0, SW_NEAR = 1, SW_MORE = 2 };

struct SphereWalk {
    const float* tab;      // the pair's FP32 sample transforms (rows of 12)
    float h, invh, L, thr, mu;
    float vr, wa, wb;      // |v_a - v_b|, |w_a|, |w_b|
    int Sn, kub;
    __device__ __forceinline__ float gap(float4 a, float4 b, int k) const
    {
        const float* T = tab + 12 * k;
        const R3<float> c = xform(T, T + 9, R3<float>{b.x, b.y, b.z});
        const float dx = c.x - a.x, dy = c.y - a.y, dz = c.z - a.z;
        return fsqrt(dx * dx + dy * dy + dz * dz) - a.w - b.w - mu;
    }
    __device__ __forceinline__ int run(float4 a, float4 b, int kf, int& ke, float& ds, int steps,
                                       unsigned& ngap) const
    {
        const float ra = fsqrt(a.x * a.x + a.y * a.y + a.z * a.z), rb = fsqrt(b.x * b.x + b.y * b.y + b.z * b.z);
        const float Ls = fminf(L, (vr + wa * ra + wb * rb) * (1.f + 1e-6f));
        const float invLs = Ls > 0.f ? 1.f / Ls : 0.f;
        for (int n = 0; n < steps; ++n) {
            const int emin = ke < 0 ? kf : ke + 1;
            int e = emin;
            if (Ls > 0.f) {
                const float ts = (float)(ke < 0 ? kf : ke) * h;
                const float need = ts + (ds - thr) * invLs;
                const float ef = floorf(fminf(need * invh, 1e6f)) - 1.f;
                e = max(emin, (int)ef);
            } else if (ke >= 0 || ds > thr) {
                return SW_CLEAR;
            }
            if (e > Sn || (e >= 1 && e - 1 >= kub)) return SW_CLEAR;
            const float g = gap(a, b, e);
            ++ngap;
            if (g <= thr) return SW_NEAR;
            ds = g;
            ke = e;
            if (e >= Sn) return SW_CLEAR;
        }
        return SW_MORE;
    }
};

__device__ __forceinline__ SphereWalk sphere_walk(const PairDev& P, const float* tab, int kub)
{
    SphereWalk w;
    w.tab = tab;
    w.Sn = P.samples;
    w.h = (float)(P.dt / w.Sn);
    w.invh = 1.f / w.h;
    w.L = (float)P.L;
    w.vr = P.vr;
    w.wa = P.wa;
    w.wb = P.wb;
    w.mu = P.mu;
    w.thr = (float)P.delta + P.mu + (float)(1e-6 * P.L * P.dt);
    w.kub = kub;
    return w;
}

// Compacted sampler, stage 1. Per kept tile pair (one wave; the pair's FP32
// sample transforms and both tiles' triangle spheres in LDS): lane j walks
// B's triangle sphere against A's tile sphere and lane i A's triangle sphere
// against B's tile sphere (TILE_STEPS steps each); the surviving (row,
// column) pairs, packed one per lane, take PAIR_STEPS steps of their own
// sphere walk. Pairs whose spheres come within the threshold go to the
// triangle walk list; pairs still undecided go to the sphere walk list
// (stage 1b), each with its last proven point. On the moving packing, 8 and
// 4 steps take 35 % less time than 2 and 2: every row or column cleared
// removes up to 64 pair walks.
constexpr int TREC_STAGE = 256;
constexpr int TILE_STEPS = 8;   // walk steps of a triangle sphere against the other tile's sphere
constexpr int PAIR_STEPS = 4;   // walk steps of a packed triangle-sphere pair in stage 1

__global__ __launch_bounds__(64) void k_toi_near(const PairDev* __restrict__ pairs, TriStore S,
                                                 const float* __restrict__ table,
                                                 const ToiItem* __restrict__ items, int64_t item_total,
                                                 int32_t* queue, const int32_t* __restrict__ pair_kub,
                                                 ToiRec* __restrict__ trecs, int32_t* trec_count, int64_t trec_cap,
                                                 ToiRec* __restrict__ srecs, int32_t* srec_count, int64_t srec_cap,
                                                 unsigned long long* stat)
{
    unsigned ngap = 0;
    unsigned long long nkept = 0, ntiled = 0;
    __shared__ float tab[MAX_ROWS * 12];
    __shared__ float4 asph[TILE], bsph[TILE];
    __shared__ uint8_t rows[TILE], cols[TILE];
    __shared__ ToiRec tstage_buf[TREC_STAGE];
    __shared__ ToiRec sstage_buf[TREC_STAGE];
    WaveStage<ToiRec, TREC_STAGE> tst{tstage_buf, 0}, sst{sstage_buf, 0};
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    XcdQueue<16> wq;
    wq.init(queue, (int)item_total);
    int tab_pair = -1;   // pair whose sample table is in LDS
    for (;;) {
        // a chunk of the item list, one item per lane; culled tile pairs are skipped
        int cnt = 0;
        const int b0 = wq.take(16, cnt);
        if (cnt == 0) break;
        ToiItem mine{0, 0, -1, 0.f};
        if (lane < cnt) mine = items[b0 + lane];
        uint64_t kept = __ballot(mine.kfirst >= 0);
        while (kept) {
            const int src = __ffsll((unsigned long long)kept) - 1;
            kept &= kept - 1;
            const ToiItem w{__builtin_amdgcn_readlane(mine.pair, src), __builtin_amdgcn_readlane(mine.tiles, src),
                            __builtin_amdgcn_readlane(mine.kfirst, src),
                            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.dlb), src))};
            const PairDev& P = pairs[w.pair];
            const int ta = w.tiles >> 16, tb = w.tiles & 0xffff;
            const int Sn = P.samples, kf = w.kfirst;
            ++nkept;
            ntiled += (unsigned long long)(min(TILE, P.na - ta * TILE) * min(TILE, P.nb - tb * TILE));
            if (w.pair != tab_pair) {   // consecutive items mostly share their pair's table
                for (int i = lane; i < (Sn + 1) * 12; i += TILE) tab[i] = table[P.table0 * 12 + i];
                tab_pair = w.pair;
            }
            const int ia = ta * TILE + lane;
            const int nbt = min(TILE, P.nb - tb * TILE);
            const float4 bl = S.tri_sph[P.tri0_b + min(tb * TILE + lane, P.nb - 1)];
            bsph[lane] = bl;
            const float4 as = S.tri_sph[P.tri0_a + min(ia, P.na - 1)];
            const float4 tsa = S.tile_sph[P.tile0_a + ta], tsb = S.tile_sph[P.tile0_b + tb];
            __syncthreads();
            const SphereWalk sw = sphere_walk(P, tab, __atomic_load_n(&pair_kub[w.pair], __ATOMIC_RELAXED));
            int ke = -1;
            float ds = fmaxf(w.dlb, sw.gap(tsa, bl, kf));
            const bool jnear = lane < nbt && sw.run(tsa, bl, kf, ke, ds, TILE_STEPS, ngap) != SW_CLEAR;
            ke = -1;
            ds = fmaxf(w.dlb, sw.gap(as, tsb, kf));
            const bool a_on = ia < P.na && sw.run(as, tsb, kf, ke, ds, TILE_STEPS, ngap) != SW_CLEAR;
            ngap += 2;
            // surviving rows (A triangles) and columns (B triangles), packed one
            // (row, column) pair per lane
            const uint64_t jm = __ballot(jnear), im = __ballot(a_on);
            asph[lane] = as;
            if (jnear) cols[__popcll(jm & below)] = (uint8_t)lane;
            if (a_on) rows[__popcll(im & below)] = (uint8_t)lane;
            __syncthreads();
            const int ni = __popcll(im), nj = __popcll(jm), np = ni * nj;
            // q / nj through the reciprocal: exact for q < 4096 and nj <= 64
            const float rnj = nj > 0 ? 1.f / (float)nj : 0.f;
            for (int q0 = 0; q0 < np; q0 += TILE) {
                const int q = q0 + lane;
                int r = SW_CLEAR, i = 0, j = 0;
                ke = -1;
                ds = 0.f;
                if (q < np) {
                    const int a = (int)(((float)q + 0.5f) * rnj);
                    i = rows[a];
                    j = cols[q - a * nj];
                    const float4 x = asph[i], b = bsph[j];
                    ds = fmaxf(w.dlb, sw.gap(x, b, kf));
                    r = sw.run(x, b, kf, ke, ds, PAIR_STEPS, ngap);
                    ++ngap;
                }
                const ToiRec rec{(uint32_t)w.pair, ((uint32_t)(ta * TILE + i) << 16) | (uint32_t)(tb * TILE + j),
                                 (int16_t)kf, (int16_t)ke, ds};
                tst.push(r == SW_NEAR, rec);
                tst.maybe_flush(trecs, trec_count, trec_cap);
                sst.push(r == SW_MORE, rec);
                sst.maybe_flush(srecs, srec_count, srec_cap);
            }
            __syncthreads();
        }
    }
    tst.flush(trecs, trec_count, trec_cap);
    sst.flush(srecs, srec_count, srec_cap);
    unsigned long long g = ngap;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
    put_wave_stat(stat, g);
    put_wave_stat(stat + 2 * STAT_WAVES, nkept);    // wave-uniform
    put_wave_stat(stat + 3 * STAT_WAVES, ntiled);   // wave-uniform
}

// Stage 1b: the sphere walks still undecided after stage 1, one per lane;
// idle lanes are refilled together from the list (as in stage 2). Walks that
// come within the threshold go to the triangle walk list.
__global__ __launch_bounds__(64) void k_toi_swalk(const PairDev* __restrict__ pairs, TriStore S,
                                                  const float* __restrict__ table,
                                                  const ToiRec* __restrict__ srecs,
                                                  const int32_t* __restrict__ srec_count, int64_t srec_cap,
                                                  int32_t* queue, const int32_t* __restrict__ pair_kub,
                                                  ToiRec* __restrict__ trecs, int32_t* trec_count, int64_t trec_cap,
                                                  unsigned long long* gap_slots)
{
    unsigned ngap = 0;
    __shared__ ToiRec stage_buf[TREC_STAGE];
    WaveStage<ToiRec, TREC_STAGE> st{stage_buf, 0};
    const int lane = lane_id();
    const int n = (int)min((int64_t)srec_count[0], srec_cap);
    XcdQueue<256> wq;
    wq.init(queue, n);
    bool valid = false;
    ToiRec r{0, 0, 0, 0, 0.f};
    float4 as = make_float4(0.f, 0.f, 0.f, 0.f), bs = as;
    SphereWalk sw{};
    int ke = -1;
    float ds = 0.f;
    for (;;) {
        const uint64_t idle = __ballot(!valid);
        const int nidle = __popcll(idle);
        if (nidle >= 16) {
            const bool was_idle = !valid;
            const int rank = __popcll(idle & ((1ull << lane) - 1ull));
            int filled = 0;
            while (filled < nidle) {
                int cnt = 0;
                const int b = wq.take(nidle - filled, cnt);
                if (cnt == 0) break;
                if (was_idle && rank >= filled && rank < filled + cnt) {
                    r = srecs[b + rank - filled];
                    const PairDev& P = pairs[r.pair];
                    as = S.tri_sph[P.tri0_a + (int)(r.ij >> 16)];
                    bs = S.tri_sph[P.tri0_b + (int)(r.ij & 0xffffu)];
                    sw = sphere_walk(P, table + P.table0 * 12, __atomic_load_n(&pair_kub[r.pair], __ATOMIC_RELAXED));
                    ke = r.ke;
                    ds = r.ds;
                    valid = true;
                }
                filled += cnt;
            }
            if (__ballot(valid) == 0) break;
        }
        bool go = false;
        if (valid) {
            const int res = sw.run(as, bs, r.kf, ke, ds, 4, ngap);
            if (res != SW_MORE) valid = false;
            go = res == SW_NEAR;
        }
        st.push(go, ToiRec{r.pair, r.ij, r.kf, (int16_t)ke, ds});
        st.maybe_flush(trecs, trec_count, trec_cap);
    }
    st.flush(trecs, trec_count, trec_cap);
    unsigned long long g = ngap;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
    put_wave_stat(gap_slots, g);
}

// Compacted sampler, stage 2: every lane walks the intervals of its own
// triangle pair (the interval logic of the oracle's scan, on FP32 samples
// with margin mu). A lane whose walk ends takes the next pair of the list:
// when half of the wave is idle, the idle lanes are refilled together from
// the wave's chunk of the list, so lanes stay busy although walks differ in
// length. An interval that cannot be cleared is handed to the FP64 end-game.
constexpr int WALK_REFILL = 32;

template <typename T>
__global__ __launch_bounds__(64) void k_toi_walk(const PairDev* __restrict__ pairs, TriStore S,
                                                 const T* __restrict__ table,
                                                 const ToiRec* __restrict__ recs,
                                                 const int32_t* __restrict__ rec_count, int64_t rec_cap,
                                                 int32_t* queue, int32_t* pair_kub, Cand* __restrict__ eg,
                                                 int32_t* eg_count, int64_t eg_cap,
                                                 unsigned long long* sample_slots)
{
    __shared__ Cand stage_buf[CAND_STAGE];
    WaveStage<Cand, CAND_STAGE> st{stage_buf, 0};
    const int lane = lane_id();
    const int n = (int)min((int64_t)rec_count[0], rec_cap);
    XcdQueue<256> wq;
    wq.init(queue, n);
    unsigned long long evals = 0;
    bool valid = false;
    // lane state: its triangle pair, the pair's constants, the walk position
    PTri<T> A;
    R3<T> b0, b1, b2;
    int pair = 0, Sn = 0, ke = -1, kf = 0;
    int32_t sa = 0, sb = 0;
    int64_t row0 = 0;
    T mu = 0, corr = 0, delta = 0, L = 0, h = 0, slack = 0, thr = 0, ts = 0, ds = 0;
    for (;;) {
        const uint64_t idle = __ballot(!valid);
        const int nidle = __popcll(idle);
        if (nidle >= WALK_REFILL) {
            const bool was_idle = !valid;
            const int rank = __popcll(idle & ((1ull << lane) - 1ull));
            int filled = 0;
            while (filled < nidle) {
                int cnt = 0;
                const int b = wq.take(nidle - filled, cnt);
                if (cnt == 0) break;
                if (was_idle && rank >= filled && rank < filled + cnt) {
                    const ToiRec r = recs[b + rank - filled];
                    pair = (int)r.pair;
                    const PairDev& P = pairs[pair];
                    sa = P.tri0_a + (int)(r.ij >> 16);
                    sb = P.tri0_b + (int)(r.ij & 0xffffu);
                    R3<T> a0, a1, a2;
                    load_tri_packed(S, sa, a0, a1, a2);
                    A = prep(a0, a1, a2);
                    load_tri_packed(S, sb, b0, b1, b2);
                    Sn = P.samples;
                    row0 = P.table0;
                    mu = sizeof(T) == 4 ? (T)P.mu : (T)P.mu64;
                    corr = sizeof(T) == 4 ? (T)P.corr : (T)P.corr64;
                    delta = (T)P.delta;
                    L = (T)P.L;
                    h = (T)(P.dt / Sn);
                    slack = (T)(1e-6 * P.L * P.dt);
                    thr = delta + mu + slack;
                    kf = r.kf;
                    ke = r.ke;       // -1: ds bounds the distance at kf; else at sample ke
                    ts = (T)(ke < 0 ? kf : ke) * h;
                    ds = (T)r.ds;
                    valid = true;
                }
                filled += cnt;
            }
            if (__ballot(valid) == 0) break;
        }
        bool emit = false;
        int ek = 0;
        if (valid) {
            const int emin = ke < 0 ? kf : ke + 1;
            int e = emin;
            if (L > (T)0) {
                const T need = ts + (ds - thr) / L;
                const T ef = floor(fmin(need / h, (T)1e6)) - (T)1;
                e = max(emin, (int)ef);
            } else if (ke >= 0 || ds > thr) {
                e = Sn + 1;
            }
            const int kub = __atomic_load_n(&pair_kub[pair], __ATOMIC_RELAXED);
            if (e > Sn || (e >= 1 && e - 1 >= kub)) {
                valid = false;
            } else {
                T dlb, dub;
                bool xs;
                sample_eval(A, table + (row0 + e) * 12, b0, b1, b2, mu, corr, dlb, dub, xs);
                ++evals;
                const T te = (T)e * h;
                if (e == 0) {
                    if (dlb <= thr) { emit = true; ek = 0; valid = false; }
                    else { ts = 0; ds = dlb; ke = 0; }
                } else {
                    if (!xs && dub + mu + slack < delta) atomicMin(&pair_kub[pair], e);
                    if (dlb <= thr || (ds + dlb - (T)2 * (mu + slack) - L * (te - ts)) * (T)0.5 <= delta) {
                        emit = true; ek = e - 1; valid = false;
                    } else {
                        ts = te; ds = dlb; ke = e;
                        if (e >= Sn) valid = false;
                    }
                }
            }
        }
        st.push(emit, Cand{pair, sa, sb, (float)ek});
        st.maybe_flush(eg, eg_count, eg_cap);
    }
    st.flush(eg, eg_count, eg_cap);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) evals += __shfl_xor(evals, o);
    put_wave_stat(sample_slots, evals);
}

// A span of the halving recursion: its ends, their distances and lattice
// codes; h: its heap index in the subtree evaluated in round gen (0: none).
struct Span {
    double lo, hi, dlo, dhi;
    int32_t clo, chi;
    int32_t h, gen;
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

// FP64 end-game: the exact interval logic (section 5, narrowing and the
// widening remark) from the handed-over interval on, with the same result as
// one lane scanning the intervals in order. A group of EG lanes takes one
// candidate triangle pair:
//  - SCAN: the lanes evaluate EG consecutive sample times at once; interval k
//    (between lanes) is in contact at its right end, needs the halving
//    recursion (its envelope reaches delta), or is clear; the first interval
//    in order that is not clear decides, as in the sequential scan. The
//    window's distances stay in LDS, so after a graze recursion runs empty
//    the scan resumes inside the window without evaluating again;
//  - BISECT: the lanes evaluate the EG-1 midpoints of the next log2(EG)
//    levels of the bisection tree (each computed by the same halving
//    arithmetic as the sequential loop), then the group replays the path of
//    the sequential bisection through them;
//  - GRAZE: the halving recursion of one interval, depth first, left half
//    first, its stack of spans in LDS. Each round the lanes evaluate the
//    EG-1 midpoints of the next log2(EG) levels below the span on top of the
//    stack; the group's first lane then runs the sequential recursion
//    through them until it needs a midpoint outside that subtree, which
//    roots the next round. A sub-span in contact at its right end goes to
//    BISECT; when the stack runs empty the scan resumes after the interval.
// Every mode evaluates through one shared call, so a wave whose groups are in
// different modes still runs one distance evaluation per round.
// Intervals that cannot beat the pair's current best key are not scanned.
constexpr int EG = 16;
constexpr int GRAZE_DEPTH = 32;   // spans on a group's halving stack (the lattice bounds the depth)
enum { EG_SCAN = 0, EG_BISECT = 1, EG_GRAZE = 2, EG_DONE = 3 };

__global__ __launch_bounds__(64) void k_toi_endgame(const PairDev* __restrict__ pairs, TriStore S,
                                                    const Cand* __restrict__ eg,
                                                    const int32_t* __restrict__ eg_count,
                                                    int64_t eg_cap, uint64_t* pair_key,
                                                    ToiOut* __restrict__ out,
                                                    unsigned long long* stat, int from_zero)
{
    const int lane = lane_id(), r = lane & (EG - 1), gbase = lane & ~(EG - 1), g = lane / EG;
    const int64_t n = min((int64_t)eg_count[0], eg_cap);
    constexpr int GPW = TILE / EG;   // candidates per wave
    __shared__ Span gstack[GPW][GRAZE_DEPTH];
    __shared__ double gdist[GPW][EG];   // distances at the evaluated subtree's midpoints
    __shared__ double gwin[GPW][EG];    // distances at the scan window's samples
    unsigned long long evals = 0, grazes = 0;
    for (int64_t e0 = (int64_t)blockIdx.x * GPW; e0 < n; e0 += (int64_t)gridDim.x * GPW) {
        const int64_t e = e0 + g;
        int mode = e < n ? EG_SCAN : EG_DONE;
        const Cand c = eg[e < n ? e : n - 1];
        const PairDev& P = pairs[c.pair];
        R3<double> a0, a1, a2, b0, b1, b2;
        load_tri_packed(S, c.ta, a0, a1, a2);
        load_tri_packed(S, c.tb, b0, b1, b2);
        const PTri<double> A = prep(a0, a1, a2);
        const uint64_t ij = ((uint64_t)(uint32_t)S.orig[c.ta] << 16) | (uint32_t)S.orig[c.tb];
        const int k0 = from_zero ? 0 : (int)c.t;
        const int Sn = P.samples;
        const double dt = P.dt, tol = P.tol, L = P.L, delta = P.delta;
        int w0 = k0, kcur = 0, sp = 0, ggen = 0;
        int sfrom = k0;        // intervals of the window before sfrom are known clear
        bool reuse = false;    // the window's distances are in gwin (after a graze ran empty)
        double lo = 0, hi = 0, dlo = 0, dhi = 0;
        int32_t clo = 0, chi = 0;
        uint64_t rkey = ~0ull;
        double rt = 0.0;
        while (__ballot(mode != EG_DONE)) {
            // the time this lane evaluates, if any
            double tq = 0.0, d = 0.0;
            bool need = false;
            int gstate = 0;   // GRAZE, first lane: 0 next root chosen, 1 contact span found, 2 stack empty
            if (mode == EG_SCAN && !reuse) {
                const int k = w0 + r;
                if (k <= Sn) { tq = sample_time(k, dt, Sn); need = true; }
            } else if (mode == EG_BISECT || mode == EG_GRAZE) {
                // heap node r (1..EG-1) below [lo, hi] (GRAZE: the subtree's root span)
                if (r > 0) {
                    double a = lo, b = hi;
                    const int depth = 31 - __clz(r);
                    bool node_ok = true;
                    for (int lv = depth - 1; lv >= 0 && node_ok; --lv) {
                        if (__dsub_rn(b, a) <= tol) { node_ok = false; break; }
                        const double m = __dmul_rn(__dadd_rn(a, b), 0.5);
                        if ((r >> lv) & 1) a = m; else b = m;
                    }
                    if (node_ok && __dsub_rn(b, a) <= tol) node_ok = false;
                    if (node_ok) { tq = __dmul_rn(__dadd_rn(a, b), 0.5); need = true; }
                }
            }
            if (need) {
                d = dist_at(P, A, b0, b1, b2, tq);
                ++evals;
            }
            if (mode == EG_GRAZE) gdist[g][r] = d;
            if (mode == EG_SCAN) {
                if (reuse) d = gwin[g][r];
                else gwin[g][r] = d;
            }
            __syncthreads();   // one wave per block: orders the LDS writes before the reads below
            if (mode == EG_GRAZE && r == 0) {
                // the sequential recursion through this round's midpoints
                gstate = 2;
                while (sp > 0) {
                    Span s = gstack[g][--sp];
                    if (s.dhi <= delta) {
                        lo = s.lo; hi = s.hi; dlo = s.dlo; dhi = s.dhi; clo = s.clo; chi = s.chi;
                        gstate = 1;
                        break;
                    }
                    const double env = __dmul_rn(__dsub_rn(__dadd_rn(s.dlo, s.dhi),
                                                           __dmul_rn(L, __dsub_rn(s.hi, s.lo))), 0.5);
                    if (env > delta) continue;
                    if (__dsub_rn(s.hi, s.lo) <= tol) { ++grazes; continue; }
                    if (s.gen != ggen || s.h == 0) {
                        // its midpoint was not evaluated: it roots the next round
                        s.h = 1;
                        s.gen = ggen + 1;
                        gstack[g][sp++] = s;
                        lo = s.lo; hi = s.hi;
                        gstate = 0;
                        break;
                    }
                    const double mid = __dmul_rn(__dadd_rn(s.lo, s.hi), 0.5);
                    const double dm = gdist[g][s.h];
                    const int32_t cm = (s.clo + s.chi) >> 1;
                    if (sp + 2 > GRAZE_DEPTH) { ++grazes; continue; }
                    const int32_t hr = 2 * s.h + 1 < EG ? 2 * s.h + 1 : 0, hl = 2 * s.h < EG ? 2 * s.h : 0;
                    gstack[g][sp++] = Span{mid, s.hi, dm, s.dhi, cm, s.chi, hr, ggen};
                    gstack[g][sp++] = Span{s.lo, mid, s.dlo, dm, s.clo, cm, hl, ggen};
                }
            }
            // group decisions (every lane takes part in the shuffles)
            const double dn = __shfl(d, gbase + min(r + 1, EG - 1));
            const double d0 = __shfl(d, gbase);
            const int gs = __shfl(gstate, gbase);
            if (mode == EG_SCAN) {
                bool decided = false;
                if (w0 == 0 && !reuse) {
                    if (d0 <= delta) { rkey = ij; rt = 0.0; mode = EG_DONE; decided = true; }
                    else if (d0 - delta > L * dt) { mode = EG_DONE; decided = true; }
                }
                // interval k = w0 + r between this lane's point and the next
                const int k = w0 + r;
                int cls = 0;   // 0 clear/none, 1 stop (pruned or past the step), 2 hit, 3 recursion
                if (!decided) {
                    if (r == EG - 1 || k >= Sn) {
                        cls = k >= Sn ? 1 : 0;
                    } else if (k < sfrom) {
                        cls = 0;   // cleared before (its graze recursion ran empty)
                    } else {
                        const uint64_t best = __atomic_load_n(&pair_key[c.pair], __ATOMIC_RELAXED);
                        if ((best >> 32) < (((uint64_t)k << LATTICE_BITS) + 1)) {
                            cls = 1;
                        } else if (dn <= delta) {
                            cls = 2;
                        } else {
                            const double t0 = sample_time(k, dt, Sn), t1 = sample_time(k + 1, dt, Sn);
                            const double env = __dmul_rn(__dsub_rn(__dadd_rn(d, dn), __dmul_rn(L, __dsub_rn(t1, t0))), 0.5);
                            if (env <= delta) cls = __dsub_rn(t1, t0) <= tol ? 4 : 3;
                        }
                    }
                }
                const uint64_t ev = __ballot(cls == 1 || cls == 2 || cls == 3);
                const uint32_t gm = (uint32_t)((ev >> gbase) & ((1ull << EG) - 1ull));
                const int first = gm ? __ffs(gm) - 1 : EG;
                if (cls == 4 && r < first) ++grazes;   // leaf graze before the deciding interval
                const int fcls = __shfl(cls, gbase + min(first, EG - 1));
                const double fd = __shfl(d, gbase + min(first, EG - 1));
                const double fdn = __shfl(dn, gbase + min(first, EG - 1));
                if (!decided) {
                    if (first == EG) {
                        w0 += EG - 1;
                        sfrom = w0;
                        reuse = false;
                        if (w0 >= Sn) mode = EG_DONE;
                    } else if (fcls == 1) {
                        mode = EG_DONE;
                    } else {
                        kcur = w0 + first;
                        lo = sample_time(kcur, dt, Sn);
                        hi = sample_time(kcur + 1, dt, Sn);
                        dlo = fd;
                        dhi = fdn;
                        clo = 0;
                        chi = 1 << LATTICE_BITS;
                        mode = fcls == 2 ? EG_BISECT : EG_GRAZE;
                        if (mode == EG_GRAZE && r == 0) {
                            gstack[g][0] = Span{lo, hi, dlo, dhi, clo, chi, 1, ggen};
                            sp = 1;
                        }
                    }
                }
            } else if (mode == EG_BISECT) {
                // replay the sequential bisection through the evaluated nodes
                int node = 1;
                for (int lv = 0; lv < 31 && node < EG; ++lv) {
                    if (__dsub_rn(hi, lo) <= tol) break;
                    const double m = __dmul_rn(__dadd_rn(lo, hi), 0.5);
                    const int32_t cm = (clo + chi) >> 1;
                    const double dm = __shfl(d, gbase + node);
                    if (dm <= delta) { hi = m; chi = cm; node = 2 * node; }
                    else { lo = m; clo = cm; node = 2 * node + 1; }
                }
                if (__dsub_rn(hi, lo) <= tol) {
                    rkey = ((((uint64_t)kcur << LATTICE_BITS) + (uint64_t)chi) << 32) | ij;
                    rt = hi;
                    mode = EG_DONE;
                }
            } else if (mode == EG_GRAZE) {
                ++ggen;
                if (gs == 0) {             // next subtree root
                    lo = __shfl(lo, gbase); hi = __shfl(hi, gbase);
                } else if (gs == 1) {
                    lo = __shfl(lo, gbase); hi = __shfl(hi, gbase);
                    dlo = __shfl(dlo, gbase); dhi = __shfl(dhi, gbase);
                    clo = __shfl(clo, gbase); chi = __shfl(chi, gbase);
                    mode = EG_BISECT;
                } else {
                    // resume the scan after the interval; its window's
                    // distances are reused while it still covers the next one
                    const int next = kcur + 1;
                    if (next >= Sn) {
                        mode = EG_DONE;
                    } else {
                        mode = EG_SCAN;
                        sfrom = next;
                        reuse = next <= w0 + EG - 2;
                        if (!reuse) w0 = next;
                    }
                }
            }
        }
        if (e < n && r == 0) {
            if (rkey != ~0ull) atomicMin((unsigned long long*)&pair_key[c.pair], (unsigned long long)rkey);
            out[e] = ToiOut{rkey, rt};
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        evals += __shfl_xor(evals, o);
        grazes += __shfl_xor(grazes, o);
    }
    put_wave_stat(stat, evals);
    put_wave_stat(stat + STAT_WAVES, grazes);
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
// particle pair, at the pair's stored transform: (ij[2p], ij[2p + 1]), or
// the pair's time-stamp key's (i, j) when keys are given (key ~0: none).
__global__ __launch_bounds__(64) void k_pair_eval(const PairDev* __restrict__ pairs, int32_t npairs,
                                                  TriStore S, const int32_t* __restrict__ ij,
                                                  const uint64_t* __restrict__ keys, PairOut* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const PairDev& P = pairs[p];
    int io, jo;
    if (keys) {
        const uint64_t k = keys[p];
        io = k == ~0ull ? -1 : (int)((k >> 16) & 0xffff);
        jo = k == ~0ull ? -1 : (int)(k & 0xffff);
    } else {
        io = ij[2 * p];
        jo = ij[2 * p + 1];
    }
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
    load_tri_packed(S, sa, a0, a1, a2);
    load_tri_packed(S, sb, b0, b1, b2);
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
                            float* table32, double* table64)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_toi_table, dim3(blocks_for((int64_t)npairs * rows, 128, 8192)), dim3(128), 0,
                       L.stream, pairs, npairs, rows, table32, table64);
    return hipGetLastError();
}

hipError_t launch_toi_cull(const Launch& L, const PairDev* pairs, int32_t npairs, const TriStore& S,
                           const float* table, ToiItem* items)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_toi_cull, dim3(npairs), dim3(256), 0, L.stream, pairs, S, table, items);
    return hipGetLastError();
}

hipError_t launch_toi_spheres(const Launch& L, const PairDev* pairs, const TriStore& S, const float* table32,
                              const ToiItem* items, int64_t nitems,
                              int32_t* queues, const int32_t* pair_kub, ToiRec* trecs, int32_t* trec_count,
                              int64_t trec_cap, ToiRec* srecs, int32_t* srec_count, int64_t srec_cap,
                              unsigned long long* stat, int grid)
{
    hipLaunchKernelGGL(k_toi_near, dim3(grid), dim3(64), 0, L.stream, pairs, S, table32, items,
                       nitems, queues, pair_kub, trecs, trec_count, trec_cap, srecs, srec_count,
                       srec_cap, stat);
    hipLaunchKernelGGL(k_toi_swalk, dim3(grid), dim3(64), 0, L.stream, pairs, S, table32, srecs,
                       srec_count, srec_cap, queues + XCD_QUEUES * XCD_QSTRIDE, pair_kub, trecs, trec_count,
                       trec_cap, stat + STAT_WAVES);
    return hipGetLastError();
}

hipError_t launch_toi_walk(const Launch& L, const PairDev* pairs, const TriStore& S, const float* table32,
                           const double* table64, int fp64, const ToiRec* trecs, const int32_t* trec_count,
                           int64_t trec_cap, int32_t* queues, int32_t* pair_kub, Cand* eg, int32_t* eg_count,
                           int64_t eg_cap, unsigned long long* sample_slots, int grid)
{
    if (fp64)
        hipLaunchKernelGGL(k_toi_walk<double>, dim3(grid), dim3(64), 0, L.stream, pairs, S, table64,
                           trecs, trec_count, trec_cap, queues, pair_kub, eg, eg_count, eg_cap, sample_slots);
    else
        hipLaunchKernelGGL(k_toi_walk<float>, dim3(grid), dim3(64), 0, L.stream, pairs, S, table32,
                           trecs, trec_count, trec_cap, queues, pair_kub, eg, eg_count, eg_cap, sample_slots);
    return hipGetLastError();
}

hipError_t launch_toi_endgame(const Launch& L, const PairDev* pairs, const TriStore& S,
                              const Cand* eg, const int32_t* eg_count, int64_t eg_cap,
                              uint64_t* pair_key, ToiOut* out, unsigned long long* stat,
                              int from_zero, int grid)
{
    hipLaunchKernelGGL(k_toi_endgame, dim3(grid), dim3(64), 0, L.stream,
                       pairs, S, eg, eg_count, eg_cap, pair_key, out, stat, from_zero);
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
                            const TriStore& S, const int32_t* ij, PairOut* out, const uint64_t* keys)
{
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_eval, dim3((npairs + 63) / 64), dim3(64), 0, L.stream, pairs, npairs,
                       S, ij, keys, out);
    return hipGetLastError();
}

}  // namespace mcd
