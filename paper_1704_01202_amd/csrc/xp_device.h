// Device-side building blocks of the collision / ionization step (gfx950).
//
// * Elementary functions defined by the method's arithmetic contract: log, exp,
//   cbrt and sin/cos of 2 pi (k + 1/2) / 2^52, built from IEEE-754 correctly
//   rounded +, -, *, / and sqrt only.  The library is compiled with
//   -ffp-contract=off so that no product is fused into an FMA.  A bit-identical
//   result on the CPU reference is what makes long runs comparable at all: the
//   binary-collision map amplifies last-bit differences from step to step.
// * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based random
//   numbers keyed by the run seed, counter (step, cell, index, purpose<<24|sub).
// * The canonical pairwise sum of a block (leaves in slot order padded with +0
//   to a power of two, summed level by level).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xpd {

// CODATA 2018, SI
constexpr double QE = 1.602176634e-19;
constexpr double ME = 9.1093837015e-31;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double HBAR = 1.054571817e-34;
constexpr double CLIGHT = 299792458.0;
constexpr double PI = 3.141592653589793;

// Random-number purposes (word 3 of the Philox counter, << 24).
// RP_ION is one call per ion and step: word 0 decides collisional
// ionization, words 1..3 the photo events of 1s, 2s and 2p.
enum : uint32_t {
    RP_PERM_E = 1, RP_PERM_I = 2, RP_REC_I = 3, RP_REC_E = 4, RP_EE = 5,
    RP_EE_TRI = 6, RP_EI = 7, RP_ION = 8, RP_DECAY = 9, RP_DIR = 10, RP_BIN = 11,
    RP_THERM = 12, RP_REC_XS = 13, RP_PART = 14
};

__device__ __forceinline__ double bits_to_f64(uint64_t b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ uint64_t f64_to_bits(double d) { return (uint64_t)__double_as_longlong(d); }

// 2^n, -1022 <= n <= 1023
__device__ __forceinline__ double two_pow(int n) { return bits_to_f64((uint64_t)(n + 1023) << 52); }

// Natural logarithm for x > 0 (finite): reduction to m in (sqrt(1/2), sqrt(2)],
// log(1+f) = f - s (f - V), s = f / (2 + f), V = s^2 (2/3 + s^2 (2/5 + ...)).
__device__ __forceinline__ double xlog(double x)
{
    if (!(x > 0.0)) return x == 0.0 ? -__builtin_inf() : __builtin_nan("");
    if (x == __builtin_inf()) return x;
    uint64_t b = f64_to_bits(x);
    int ebias = 0;
    if ((b >> 52) == 0) {            // subnormal (sign is 0 here)
        x = x * 0x1p54;
        b = f64_to_bits(x);
        ebias = -54;
    }
    int e = (int)(b >> 52) - 1023 + ebias;
    double m = bits_to_f64((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double v = 2.0 / 23.0;
    v = 2.0 / 21.0 + z * v;
    v = 2.0 / 19.0 + z * v;
    v = 2.0 / 17.0 + z * v;
    v = 2.0 / 15.0 + z * v;
    v = 2.0 / 13.0 + z * v;
    v = 2.0 / 11.0 + z * v;
    v = 2.0 / 9.0 + z * v;
    v = 2.0 / 7.0 + z * v;
    v = 2.0 / 5.0 + z * v;
    v = 2.0 / 3.0 + z * v;
    v = z * v;
    const double l1p = f - s * (f - v);
    const double de = (double)e;
    return de * 0x1.62e42p-1 + (l1p + de * 0x1.fdf473de6af28p-22);
}

// Exponential: k = floor(x / ln2 + 1/2), r = (x - k ln2_hi) - k ln2_lo, Taylor to r^13.
__device__ __noinline__ double xexp(double x)
{
    if (x != x) return x;
    if (x > 709.78) return __builtin_inf();
    if (x < -745.14) return 0.0;
    const double k = floor(x * 0x1.71547652b82fep+0 + 0.5);
    const double r = (x - k * 0x1.62e42p-1) - k * 0x1.fdf473de6af28p-22;
    double p = 1.0 / 6227020800.0;
    p = 1.0 / 479001600.0 + r * p;
    p = 1.0 / 39916800.0 + r * p;
    p = 1.0 / 3628800.0 + r * p;
    p = 1.0 / 362880.0 + r * p;
    p = 1.0 / 40320.0 + r * p;
    p = 1.0 / 5040.0 + r * p;
    p = 1.0 / 720.0 + r * p;
    p = 1.0 / 120.0 + r * p;
    p = 1.0 / 24.0 + r * p;
    p = 1.0 / 6.0 + r * p;
    p = 0.5 + r * p;
    p = 1.0 + r * p;
    p = 1.0 + r * p;
    const int n = (int)k;
    if (n > 1023) return (p * 2.0) * two_pow(n - 1);
    if (n < -1022) return (p * two_pow(n + 600)) * two_pow(-600);
    return p * two_pow(n);
}

// Cube root for x >= 0: exponent split by 3, six Newton steps from 1 + (m'-1)/7.
__device__ __noinline__ double xcbrt(double x)
{
    if (!(x > 0.0)) return x;
    if (x == __builtin_inf()) return x;
    double post = 1.0;
    uint64_t b = f64_to_bits(x);
    if ((b >> 52) == 0) {
        x = x * 0x1p54;
        post = 0x1p-18;
        b = f64_to_bits(x);
    }
    const int e = (int)(b >> 52) - 1023;
    const int r = ((e % 3) + 3) % 3;
    const int e3 = (e - r) / 3;
    double m = bits_to_f64((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
    if (r == 1) m = m * 2.0;
    if (r == 2) m = m * 4.0;
    double y = 1.0 + (m - 1.0) * (1.0 / 7.0);
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const double t = m / (y * y);
        y = y + (t - y) / 3.0;
    }
    return (y * two_pow(e3)) * post;
}

// sin and cos of 2 pi (k + 1/2) / 2^52 for a 52-bit integer k.
__device__ __forceinline__ void xsincos2pi(uint64_t k, double& s_out, double& c_out)
{
    k &= 0x000fffffffffffffull;
    const int64_t q = (int64_t)((k + (1ull << 49)) >> 50);
    const int64_t rem = (int64_t)k - (q << 50);
    const double th = (((double)rem + 0.5) * 0x1p-50) * 0x1.921fb54442d18p+0;
    const double t2 = th * th;
    double sp = 1.0 / 355687428096000.0;
    sp = -1.0 / 1307674368000.0 + t2 * sp;
    sp = 1.0 / 6227020800.0 + t2 * sp;
    sp = -1.0 / 39916800.0 + t2 * sp;
    sp = 1.0 / 362880.0 + t2 * sp;
    sp = -1.0 / 5040.0 + t2 * sp;
    sp = 1.0 / 120.0 + t2 * sp;
    sp = -1.0 / 6.0 + t2 * sp;
    const double sn = th + th * (t2 * sp);
    double cp = 1.0 / 20922789888000.0;
    cp = -1.0 / 87178291200.0 + t2 * cp;
    cp = 1.0 / 479001600.0 + t2 * cp;
    cp = -1.0 / 3628800.0 + t2 * cp;
    cp = 1.0 / 40320.0 + t2 * cp;
    cp = -1.0 / 720.0 + t2 * cp;
    cp = 1.0 / 24.0 + t2 * cp;
    cp = -0.5 + t2 * cp;
    const double cs = 1.0 + t2 * cp;
    const int qq = (int)(q & 3);
    s_out = qq == 0 ? sn : (qq == 1 ? cs : (qq == 2 ? -sn : -cs));
    c_out = qq == 0 ? cs : (qq == 1 ? -sn : (qq == 2 ? -cs : sn));
}

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

// Uniform on (0, 1) from a 32-bit word.
__device__ __forceinline__ double u32(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

// Uniform on (0, 1) from the top 52 bits of the 64-bit word (hi, lo).
__device__ __forceinline__ double u52(uint32_t hi, uint32_t lo)
{
    const uint64_t a = ((uint64_t)hi << 32) | lo;
    return ((double)(a >> 12) + 0.5) * 0x1p-52;
}

__device__ __forceinline__ int ilog2_ceil(int n)
{
    int b = 0;
    while ((1 << b) < n) ++b;
    return b;
}

// Cross-lane moves within a wave on the VALU (DPP): CTRL is the dpp_ctrl code
// (quad permutations 0x00-0xff, row shifts 0x101-0x11f, row mirror 0x140,
// half-row mirror 0x141).  Every source lane used here lies inside the row.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
// As dpp32, with 0 in lanes whose source lies outside the row.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32z(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    const uint32_t lo = dpp32<CTRL>((uint32_t)v), hi = dpp32<CTRL>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) { return bits_to_f64(dpp64<CTRL>(f64_to_bits(v))); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Canonical pairwise sum of the 64 lanes' values (lane = leaf), returned to
// every lane.  Levels 1 and 2 pair lane l with l ^ 1 and l ^ 2; after them
// every aligned block of 4 lanes holds its node, so the mirror within a half
// row (8 lanes) and within a row (16 lanes) meet the sibling node exactly as
// l ^ 4 and l ^ 8 would.  The four row sums are then added as
// (r0 + r1) + (r2 + r3).  Addition is commutative in IEEE-754, so every lane
// holds the same bits as the tree evaluated in slot order.
__device__ __forceinline__ double wave_tree_sum64(double acc)
{
    acc = acc + dpp_f64<0xb1>(acc);     // quad_perm [1,0,3,2]: lane ^ 1
    acc = acc + dpp_f64<0x4e>(acc);     // quad_perm [2,3,0,1]: lane ^ 2
    acc = acc + dpp_f64<0x141>(acc);    // half-row mirror: the other block of 4
    acc = acc + dpp_f64<0x140>(acc);    // row mirror: the other block of 8
    const uint64_t b = f64_to_bits(acc);
    const double r0 = bits_to_f64(readlane64(b, 0)), r1 = bits_to_f64(readlane64(b, 16));
    const double r2 = bits_to_f64(readlane64(b, 32)), r3 = bits_to_f64(readlane64(b, 48));
    return (r0 + r1) + (r2 + r3);
}

// Sum of the 64 lanes' integers (any order), returned to every lane.
__device__ __forceinline__ long long wave_isum64(long long v)
{
    v += (long long)dpp64<0xb1>((uint64_t)v);
    v += (long long)dpp64<0x4e>((uint64_t)v);
    v += (long long)dpp64<0x141>((uint64_t)v);
    v += (long long)dpp64<0x140>((uint64_t)v);
    const uint64_t b = (uint64_t)v;
    return (long long)(readlane64(b, 0) + readlane64(b, 16) + readlane64(b, 32) + readlane64(b, 48));
}

// Canonical pairwise sum of n leaves produced by leaf(j), over a block of B
// threads (B a multiple of 64).  Leaves are padded with +0 to P = 2^k.  Rows of
// 64 consecutive leaves are owned by waves (lane = leaf mod 64): each row is
// reduced across lanes (wave_tree_sum64), which is levels 1..6 of the tree; the row sums (the
// level-6 nodes) are then reduced pairwise in LDS, out of place, level by
// level.  For P < 64 the row is padded with zeros, which adds only +0 above
// the root.  red must hold 2 * max(1, P/64) doubles; the result (+0.0) is
// returned to every thread.
template <int B, class F>
__device__ double block_tree_sum(int n, F leaf, double* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int p = 64;
    while (p < n) p <<= 1;
    const int rows = p >> 6;
    if (rows == 1) {
        double acc = 0.0;
        if (wid == 0) {
            acc = lane < n ? leaf(lane) : 0.0;
            acc = wave_tree_sum64(acc);
        }
        if (B == 64) return acc + 0.0;
        __syncthreads();
        if (threadIdx.x == 0) red[0] = acc;
        __syncthreads();
        const double r = red[0];
        __syncthreads();
        return r + 0.0;
    }
    for (int r = wid; r < rows; r += B / 64) {
        const int j = (r << 6) + lane;
        double acc = j < n ? leaf(j) : 0.0;
        acc = wave_tree_sum64(acc);
        if (lane == 0) red[r] = acc;
    }
    __syncthreads();
    double* src = red;
    double* dst = red + rows;
    for (int len = rows; len > 1; len >>= 1) {
        const int half = len >> 1;
        for (int i = threadIdx.x; i < half; i += B) dst[i] = src[2 * i] + src[2 * i + 1];
        __syncthreads();
        double* t = src;
        src = dst;
        dst = t;
    }
    const double r = src[0];
    __syncthreads();
    return r + 0.0;
}

// Three canonical pairwise sums at once, each with the tree of
// block_tree_sum: leaf(j, x, y, z) gives the three leaves of index j (+0 for
// j >= n is the caller's).  One pass over the leaves, one barrier per level
// for the three trees.  red must hold 6 * max(1, P/64) doubles; the sums (+0.0)
// are returned to every thread of a block of B threads.
template <int B, class F>
__device__ void block_tree_sum3(int n, F leaf, double* red, double& sx, double& sy, double& sz)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    int p = 64;
    while (p < n) p <<= 1;
    const int rows = p >> 6;
    if (rows == 1) {
        double x = 0.0, y = 0.0, z = 0.0;
        if (wid == 0) {
            if (lane < n) leaf(lane, x, y, z);
            x = wave_tree_sum64(x);
            y = wave_tree_sum64(y);
            z = wave_tree_sum64(z);
        }
        if (B > 64) {
            __syncthreads();
            if (tid == 0) {
                red[0] = x;
                red[1] = y;
                red[2] = z;
            }
            __syncthreads();
            x = red[0];
            y = red[1];
            z = red[2];
            __syncthreads();
        }
        sx = x + 0.0;
        sy = y + 0.0;
        sz = z + 0.0;
        return;
    }
    // component c's rows in red[2 rows c ...], ping-ponged as in block_tree_sum
    for (int r = wid; r < rows; r += B / 64) {
        const int j = (r << 6) + lane;
        double x = 0.0, y = 0.0, z = 0.0;
        if (j < n) leaf(j, x, y, z);
        x = wave_tree_sum64(x);
        y = wave_tree_sum64(y);
        z = wave_tree_sum64(z);
        if (lane == 0) {
            red[r] = x;
            red[2 * rows + r] = y;
            red[4 * rows + r] = z;
        }
    }
    __syncthreads();
    int so = 0, dof = rows;   // offsets of src and dst within a component's buffer
    for (int len = rows; len > 1; len >>= 1) {
        const int half = len >> 1;
        for (int i = tid; i < 3 * half; i += B) {
            const int c = i / half, ii = i - c * half;
            double* cb = red + 2 * rows * c;
            cb[dof + ii] = cb[so + 2 * ii] + cb[so + 2 * ii + 1];
        }
        __syncthreads();
        const int t = so;
        so = dof;
        dof = t;
    }
    sx = red[so] + 0.0;
    sy = red[2 * rows + so] + 0.0;
    sz = red[4 * rows + so] + 0.0;
    __syncthreads();
}

// Block-wide integer sum (any order).
template <int B>
__device__ long long block_isum(long long v, long long* red)
{
    v = wave_isum64(v);
    if (B == 64) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    long long s = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Stable in-order compaction helper: exclusive prefix count of pred over
// indices j = 0..n-1 processed in chunks of B (slot order), writing the
// position of every j with pred(j) through emit(j, pos).  Returns the total.
template <int B, class P, class E>
__device__ int block_ordered_select(int n, P pred, E emit, int* red)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    int base = 0;
    for (int c0 = 0; c0 < n; c0 += B) {
        const int j = c0 + tid;
        const bool f = j < n && pred(j);
        const uint64_t bal = __ballot(f);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        const int wcount = __popcll(bal);
        if (B > 64) {
            __syncthreads();
            if (lane == 0) red[wid] = wcount;
            __syncthreads();
        }
        int woff = 0, tot = wcount;
        if (B > 64) {
            tot = 0;
#pragma unroll
            for (int w = 0; w < B / 64; ++w) {
                if (w < wid) woff += red[w];
                tot += red[w];
            }
        }
        if (f) emit(j, base + woff + before);
        base += tot;
    }
    if (B > 64) __syncthreads();
    return base;
}

// Block-wide exclusive prefix sum of one value per thread, in thread order;
// the block total through total.  red: >= B / 64 entries.
template <int B, class T>
__device__ T block_exclusive_sum(T v, T* red, T& total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T incl = v;
    if constexpr (sizeof(T) == 4) {
        // inclusive scan on the VALU: shifts by 1, 2, 4, 8 within rows of 16
        // (lanes whose source lies before the row read 0), then the last lane
        // of row 0 into row 1 and of row 2 into row 3, then lane 31 into rows 2, 3
        incl += (T)dpp32z<0x111>((uint32_t)incl);
        incl += (T)dpp32z<0x112>((uint32_t)incl);
        incl += (T)dpp32z<0x114>((uint32_t)incl);
        incl += (T)dpp32z<0x118>((uint32_t)incl);
        incl += (T)__builtin_amdgcn_update_dpp(0, (int)incl, 0x142, 0xa, 0xf, false);
        incl += (T)__builtin_amdgcn_update_dpp(0, (int)incl, 0x143, 0xc, 0xf, false);
    } else {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
    }
    if (B == 64) {
        if constexpr (sizeof(T) == 4) total = (T)__builtin_amdgcn_readlane((int)incl, 63);
        else total = __shfl(incl, 63, 64);
        return incl - v;
    }
    __syncthreads();
    if (lane == 63) red[wid] = incl;
    __syncthreads();
    T woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) {
        if (w < wid) woff += red[w];
        tot += red[w];
    }
    __syncthreads();
    total = tot;
    return woff + incl - v;
}

// Bitonic sort of p = 2^k 64-bit keys in LDS (ascending), B threads.
template <int B, class P>
__device__ void bitonic_sort(P a, int p)
{
    for (int k = 2; k <= p; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < p / 2; i += B) {
                const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int hi = lo + j;
                const bool up = (lo & k) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if (up ? (x > y) : (x < y)) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// The value of lane ^ j: strides 1 and 2 by quad permutations, 4 and 8 by
// row shifts (the partner lies in the same row of 16), 16 and 32 by shuffles.
// lane: the lane index or any index with the same low four bits.
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v, int j, int lane)
{
    if (j == 1) return dpp64<0xb1>(v);
    if (j == 2) return dpp64<0x4e>(v);
    if (j == 4) {
        const uint64_t dn = dpp64<0x114>(v), up = dpp64<0x104>(v);   // lane - 4, lane + 4
        return (lane & 4) ? dn : up;
    }
    if (j == 8) {
        const uint64_t dn = dpp64<0x118>(v), up = dpp64<0x108>(v);   // lane - 8, lane + 8
        return (lane & 8) ? dn : up;
    }
    return shfl_xor_u64(v, j);
}

__device__ __forceinline__ uint64_t shfl_xor_u64w(uint64_t v, int m, int width)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, width);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, width);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of P = W K keys held by a group of W lanes (W a power of two
// <= 64, groups aligned in the wave): element e = t + W m is key[m] of group
// lane t.  Strides below W exchange across the group's lanes, larger strides
// between a lane's own registers.  Same network as the one-wave sort.
template <int W, int K>
__device__ __forceinline__ void group_bitonic(uint64_t (&key)[K])
{
    const int t = threadIdx.x & (W - 1);
#pragma unroll
    for (int k = 2; k <= W * K; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= W) {
                const int mj = j / W;
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    if (m & mj) continue;
                    const int e = t + W * m;
                    const bool up = (e & k) == 0;
                    const uint64_t x = key[m], y = key[m | mj];
                    const bool sw = up ? (x > y) : (x < y);
                    key[m] = sw ? y : x;
                    key[m | mj] = sw ? x : y;
                }
            } else {
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const int e = t + W * m;
                    const uint64_t o = j <= 8 ? xor_lane_u64(key[m], j, t) : shfl_xor_u64w(key[m], j, W);
                    const bool up = (e & k) == 0;
                    const bool lower = (t & j) == 0;
                    const bool take_min = lower == up;
                    const bool less = o < key[m];
                    key[m] = (take_min == less) ? o : key[m];
                }
            }
        }
    }
}

// Canonical pairwise sum over n <= 4 W leaves by a group of W lanes: leaves
// padded with +0 to p = pow2 >= n; lane t holds the aligned block of R = p / W
// leaves (R <= 4) and sums it pairwise, then the groups' lanes are summed
// pairwise by shuffles.  Equals the level-by-level sum of the p leaves.
template <int W, class F>
__device__ double group_tree_sum(int n, F leaf)
{
    const int t = threadIdx.x & (W - 1);
    int p = 1;
    while (p < n) p <<= 1;
    const int R = p <= W ? 1 : p / W;   // leaves per lane: 1, 2 or 4
    // one evaluation site for the leaf: the in-lane block is read in a loop
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        const int j = t * R + r;
        const double v = j < n ? leaf(j) : 0.0;
        if (r == 0) a0 = v;
        else if (r == 1) a1 = v;
        else if (r == 2) a2 = v;
        else a3 = v;
    }
    const double acc0 = R == 1 ? a0 : (R == 2 ? a0 + a1 : (a0 + a1) + (a2 + a3));
    double acc = acc0;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) acc = acc + __shfl_down(acc, off, W);
    return __shfl(acc, 0, W) + 0.0;
}

}  // namespace xpd
