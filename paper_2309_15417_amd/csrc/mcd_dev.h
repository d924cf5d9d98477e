// Device helpers shared by the kernel files: triangle loads, rigid
// transforms, LDS packing of prepared triangles and wave-level compaction.
#pragma once

#include <hip/hip_runtime.h>

#include "mcd_geom.h"
#include "mcd_internal.h"

namespace mcd {

static constexpr int F32_STRIDE = 9;    // float4 per LDS triangle (32 used + pad: 36 floats)
static constexpr int F64_STRIDE = 17;   // double2 per LDS triangle (32 used + pad: 34 doubles)

// Rotation matrix and position at time t of a state (x, unit q, v, w):
// q(t) = exp(t w / 2) * q0, x(t) = x0 + v t.
static __device__ __forceinline__ void pose(const double* s, double t, double* R, double* x)
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

template <typename T>
static __device__ __forceinline__ void to_array(const PTri<T>& t, T* o)
{
    o[0] = t.p0.x; o[1] = t.p0.y; o[2] = t.p0.z;
    o[3] = t.p1.x; o[4] = t.p1.y; o[5] = t.p1.z;
    o[6] = t.p2.x; o[7] = t.p2.y; o[8] = t.p2.z;
    o[9] = t.n.x; o[10] = t.n.y; o[11] = t.n.z; o[12] = t.off;
    o[13] = t.g0.x; o[14] = t.g0.y; o[15] = t.g0.z; o[16] = t.h0;
    o[17] = t.g1.x; o[18] = t.g1.y; o[19] = t.g1.z; o[20] = t.h1;
    o[21] = t.g2.x; o[22] = t.g2.y; o[23] = t.g2.z; o[24] = t.h2;
    o[25] = t.ee0; o[26] = t.ee1; o[27] = t.ee2;
    o[28] = t.ie0; o[29] = t.ie1; o[30] = t.ie2; o[31] = t.emax;
}

template <typename T>
static __device__ __forceinline__ PTri<T> from_array(const T* o)
{
    PTri<T> t;
    t.p0 = {o[0], o[1], o[2]}; t.p1 = {o[3], o[4], o[5]}; t.p2 = {o[6], o[7], o[8]};
    t.n = {o[9], o[10], o[11]}; t.off = o[12];
    t.g0 = {o[13], o[14], o[15]}; t.h0 = o[16];
    t.g1 = {o[17], o[18], o[19]}; t.h1 = o[20];
    t.g2 = {o[21], o[22], o[23]}; t.h2 = o[24];
    t.ee0 = o[25]; t.ee1 = o[26]; t.ee2 = o[27];
    t.ie0 = o[28]; t.ie1 = o[29]; t.ie2 = o[30]; t.emax = o[31];
    return t;
}

template <typename T>
static __device__ __forceinline__ void load_tri(const T* v, int64_t cap, int64_t i, R3<T>& a, R3<T>& b,
                                         R3<T>& c)
{
    a = {v[0 * cap + i], v[1 * cap + i], v[2 * cap + i]};
    b = {v[3 * cap + i], v[4 * cap + i], v[5 * cap + i]};
    c = {v[6 * cap + i], v[7 * cap + i], v[8 * cap + i]};
}

// One triangle from the packed copies (for gathers of scattered triangles:
// 48 or 80 contiguous bytes instead of one element of each of 9 planes).
static __device__ __forceinline__ void load_tri_packed(const TriStore& S, int64_t i, R3<float>& a,
                                                       R3<float>& b, R3<float>& c)
{
    const float4 x = S.p32[4 * i], y = S.p32[4 * i + 1], z = S.p32[4 * i + 2];
    a = {x.x, x.y, x.z};
    b = {x.w, y.x, y.y};
    c = {y.z, y.w, z.x};
}

// The same with the triangle's plane (unit normal n, offset off: n.x = off on
// the plane), body frame.
static __device__ __forceinline__ void load_tri_plane(const TriStore& S, int64_t i, R3<float>& a,
                                                      R3<float>& b, R3<float>& c, R3<float>& n, float& off)
{
    const float4 x = S.p32[4 * i], y = S.p32[4 * i + 1], z = S.p32[4 * i + 2], w = S.p32[4 * i + 3];
    a = {x.x, x.y, x.z};
    b = {x.w, y.x, y.y};
    c = {y.z, y.w, z.x};
    n = {z.y, z.z, z.w};
    off = w.x;
}

static __device__ __forceinline__ void load_tri_packed(const TriStore& S, int64_t i, R3<double>& a,
                                                       R3<double>& b, R3<double>& c)
{
    const double2 u = S.p64[5 * i], v = S.p64[5 * i + 1], w = S.p64[5 * i + 2], x = S.p64[5 * i + 3],
                  y = S.p64[5 * i + 4];
    a = {u.x, u.y, v.x};
    b = {v.y, w.x, w.y};
    c = {x.x, x.y, y.x};
}

template <typename T>
static __device__ __forceinline__ R3<T> xform(const T* M, const T* m, R3<T> x)
{
    return {M[0] * x.x + M[1] * x.y + M[2] * x.z + m[0],
            M[3] * x.x + M[4] * x.y + M[5] * x.z + m[1],
            M[6] * x.x + M[7] * x.y + M[8] * x.z + m[2]};
}

static __device__ __forceinline__ int lane_id() { return __lane_id(); }

static __device__ __forceinline__ int pop_item(int32_t* queue)
{
    int it = 0;
    if (lane_id() == 0) it = atomicAdd(queue, 1);
    return __shfl(it, 0);
}

// Work items taken from the queue CHUNK at a time (fewer atomics on the one
// counter): call with a per-wave cursor initialised to CHUNK.
template <int CHUNK>
static __device__ __forceinline__ int pop_chunked(int32_t* queue, int& base, int& k)
{
    if (k == CHUNK) {
        int b = 0;
        if (lane_id() == 0) b = atomicAdd(queue, CHUNK);
        base = __builtin_amdgcn_readfirstlane(b);
        k = 0;
    }
    return base + k++;
}

// Work queue split in XCD_QUEUES contiguous ranges of the item list, one
// counter each (64 bytes apart). Workgroups are dispatched round-robin over
// the 8 XCDs, so blockIdx % 8 names the XCD a wave runs on: it takes chunks
// from its own range first (items of one pair are contiguous, so that pair's
// triangles stay in this XCD's L2) and then from the other ranges. Eight
// counters instead of one also take the serialisation of same-address
// atomics off the critical path.
constexpr int XCD_QUEUES = 8;
constexpr int XCD_QSTRIDE = 16;   // int32 between counters

template <int CHUNK>
struct XcdQueue {
    int32_t* q;        // XCD_QUEUES counters, XCD_QSTRIDE apart, zero at launch
    int n;             // items
    int home, tries;   // first range, ranges tried so far
    int lo, hi;        // current range
    int base, k;       // current chunk
    int ck;            // chunk size (at most CHUNK): smaller for short lists, so that every wave gets work
    __device__ __forceinline__ void init(int32_t* queues, int nitems, int chunk = CHUNK)
    {
        q = queues;
        n = nitems;
        ck = chunk < 1 ? 1 : (chunk > CHUNK ? CHUNK : chunk);
        home = blockIdx.x % XCD_QUEUES;
        tries = 0;
        set_range();
        k = ck;
        base = hi;
    }
    __device__ __forceinline__ void set_range()
    {
        const int r = (home + tries) % XCD_QUEUES;
        lo = (int)((int64_t)n * r / XCD_QUEUES);
        hi = (int)((int64_t)n * (r + 1) / XCD_QUEUES);
    }
    // Up to `want` consecutive items: returns the first, cnt the number taken
    // (0 when every range is exhausted).
    __device__ __forceinline__ int take(int want, int& cnt)
    {
        for (;;) {
            if (k < ck && base + k < hi) {
                const int avail = min(ck - k, hi - (base + k));
                cnt = min(want, avail);
                const int r = base + k;
                k += cnt;
                return r;
            }
            if (tries >= XCD_QUEUES) { cnt = 0; return 0; }
            int b = 0;
            if (lane_id() == 0) b = atomicAdd(q + ((home + tries) % XCD_QUEUES) * XCD_QSTRIDE, ck);
            b = __builtin_amdgcn_readfirstlane(b);
            base = lo + b;
            k = 0;
            if (base >= hi) {
                ++tries;
                if (tries < XCD_QUEUES) set_range();
                k = ck;
            }
        }
    }
    // Next item index, or -1 when every range is exhausted.
    __device__ __forceinline__ int pop()
    {
        for (;;) {
            if (k < ck && base + k < hi) return base + k++;
            if (tries >= XCD_QUEUES) return -1;
            int b = 0;
            if (lane_id() == 0) b = atomicAdd(q + ((home + tries) % XCD_QUEUES) * XCD_QSTRIDE, ck);
            b = __builtin_amdgcn_readfirstlane(b);
            base = lo + b;
            k = 0;
            if (base >= hi) {
                ++tries;
                if (tries < XCD_QUEUES) set_range();
                k = ck;
            }
        }
    }
};

// Reserve slots for the lanes whose flag is set; returns this lane's slot.
static __device__ __forceinline__ int64_t reserve(bool flag, int32_t* counter)
{
    uint64_t m = __ballot(flag);
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, 0);
    return (int64_t)base + __popcll(m & ((1ull << lane_id()) - 1ull));
}

// Wave-local staging of records in LDS; flush() appends them to a global
// list with one atomic. Only for 64-thread (single-wave) blocks.
template <typename Rec, int CAP>
struct WaveStage {
    Rec* buf;
    int n;   // wave-uniform count
    __device__ __forceinline__ void push(bool flag, const Rec& r)
    {
        const uint64_t m = __ballot(flag);
        if (!m) return;
        const int pos = n + __popcll(m & ((1ull << lane_id()) - 1ull));
        if (flag) buf[pos] = r;
        n += __popcll(m);
    }
    __device__ __forceinline__ void flush(Rec* dst, int32_t* count, int64_t cap)
    {
        __syncthreads();
        int base = 0;
        if (lane_id() == 0 && n) base = atomicAdd(count, n);
        base = __shfl(base, 0);
        for (int k = lane_id(); k < n; k += 64)
            if ((int64_t)base + k < cap) dst[base + k] = buf[k];
        __syncthreads();
        n = 0;
    }
    __device__ __forceinline__ void maybe_flush(Rec* dst, int32_t* count, int64_t cap)
    {
        if (n > CAP - 64) flush(dst, count, cap);
    }
};

constexpr int CAND_STAGE = 256;   // LDS staging of candidate records per wave

// atomicMin of v into dst[key] over the lanes with flag set, one atomic per
// distinct key of the wave (lanes of a wave mostly share their key, and
// same-address atomics serialise in memory).
static __device__ __forceinline__ void wave_min_by_key(bool flag, int key, uint64_t v, uint64_t* dst)
{
    uint64_t pending = __ballot(flag);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int k = __builtin_amdgcn_readlane(key, leader);
        const bool mine = flag && key == k;
        unsigned long long m = mine ? (unsigned long long)v : ~0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long u = __shfl_xor(m, o);
            m = u < m ? u : m;
        }
        if (lane_id() == leader) atomicMin((unsigned long long*)&dst[k], m);
        pending &= ~__ballot(mine);
    }
}

// cnt[key] += (lanes with flag set and that key), one atomic per distinct
// key of the wave.
static __device__ __forceinline__ void wave_count_by_key(bool flag, int key, int32_t* cnt)
{
    uint64_t pending = __ballot(flag);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int k = __builtin_amdgcn_readlane(key, leader);
        const uint64_t same = __ballot(flag && key == k);
        if (lane_id() == leader) atomicAdd(&cnt[k], (int)__popcll(same));
        pending &= ~same;
    }
}

// A wave's partial count into its slot of a row (one wave per block).
static __device__ __forceinline__ void put_wave_stat(unsigned long long* slots, unsigned long long v)
{
    if (lane_id() == 0) slots[blockIdx.x] = v;
}

static __device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}


}  // namespace mcd
