// rng.hpp -- counter-based random streams and IEEE-exact transcendental
// helpers for the DSMC kernels.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4): ten
// rounds, each two 32x32->64 products of counter words with fixed odd
// multipliers, the high halves xored into the other words and the key, the key
// advanced by Weyl constants between rounds.
//
// Counter layout of every stream: word 0 = time step, word 1 = entity
// (particle slot, cell or particle index), word 2 = sub-index (wall-hit ordinal
// or collision candidate), word 3 = tag << 24 | call.  The key is the
// instance's 64-bit seed.  Independent instances therefore never share a
// stream, whatever group they run in.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsmc {

enum : uint32_t { kTagInit = 1u, kTagWall = 2u, kTagColl = 3u, kTagInject = 5u };

__host__ __device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32x32->64 product as one 64-bit multiply (one v_mad_u64_u32
        // on the device instead of separate low and high multiplies)
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t a = (uint32_t)pa, ah = (uint32_t)(pa >> 32);
        const uint32_t b = (uint32_t)pb, bh = (uint32_t)(pb >> 32);
        c = make_uint4(bh ^ c.y ^ k0, b, ah ^ c.w ^ k1, a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// One stream (fixed step/entity/sub/tag); next() advances the call number.
struct Stream {
    uint32_t k0, k1, step, entity, sub, tagcall;
    __device__ __forceinline__ Stream(uint32_t key0, uint32_t key1, uint32_t s, uint32_t e,
                                      uint32_t q, uint32_t tag)
        : k0(key0), k1(key1), step(s), entity(e), sub(q), tagcall(tag << 24) {}
    __device__ __forceinline__ uint4 next() {
        uint4 x = philox4x32_10(make_uint4(step, entity, sub, tagcall), k0, k1);
        tagcall += 1u;
        return x;
    }
};

// ---------------------------------------------------------------- FP64
// Uniform on (0, 1]: 27 high bits of one word and 26 of the next form k in
// [0, 2^53); U = (k + 1) 2^-53, exact and never zero.
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
    const uint64_t k = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return (double)(k + 1ull) * 0x1p-53;
}

// ln(u) for u in (0, 1] using only IEEE add/mul/div: u = 2^e m with m in
// [1/sqrt2, sqrt2]; ln m = 2 atanh(s), s = (m - 1)/(m + 1); the odd series
// 2 s sum_i z^i / (2i + 1), z = s^2, is summed by Horner from i = 11 down.
// The same operation sequence as the host recipe gives identical bits.
__device__ __forceinline__ double series_log(double u) {
#pragma clang fp contract(off)
    const uint64_t bits = (uint64_t)__double_as_longlong(u);
    int ex = (int)((bits >> 52) & 0x7FFull) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                                0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        ex += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
#pragma unroll
    for (int i = 10; i >= 0; --i) p = p * z + 1.0 / (double)(2 * i + 1);
    return (double)ex * 0x1.62e42fefa39efp-1 + (s * p) * 2.0;
}

// ---------------------------------------------------------------- FP32
// Uniform on (0, 1] from the top 24 bits of a word.
__device__ __forceinline__ float u24(uint32_t x) {
    return (float)((x >> 8) + 1u) * 0x1p-24f;
}

// Precision-dependent pieces of the recipe.  The FP64 specialisation is the
// exact recipe (53-bit uniforms, series log, correctly rounded division and
// square root); the FP32 one is the fast mode's: 24-bit uniforms and the
// hardware's single-instruction reciprocal, square root and logarithm (each
// within about one ulp).
template <class R> struct Num;

template <> struct Num<double> {
    __device__ __forceinline__ static void uni2(const uint4& x, double& a, double& b) {
        a = u53(x.x, x.y);
        b = u53(x.z, x.w);
    }
    __device__ __forceinline__ static double log(double u) { return series_log(u); }
    __device__ __forceinline__ static double sqrt(double v) { return __builtin_sqrt(v); }
    __device__ __forceinline__ static double div(double a, double b) { return a / b; }
};

template <> struct Num<float> {
    __device__ __forceinline__ static void uni2(const uint4& x, float& a, float& b) {
        a = u24(x.x);
        b = u24(x.z);
    }
    // v_log_f32 is the base-2 logarithm
    __device__ __forceinline__ static float log(float u) {
        return __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    }
    __device__ __forceinline__ static float sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
    __device__ __forceinline__ static float div(float a, float b) {
        return a * __builtin_amdgcn_rcpf(b);
    }
};

// Marsaglia-Bray polar method: a pair of independent normals with standard
// deviation sd, drawing calls from the stream until 0 < a^2 + b^2 < 1.
template <class R>
__device__ __forceinline__ void normal_pair(Stream& st, R sd, R& n0, R& n1) {
#pragma clang fp contract(off)
    for (;;) {
        R ua, ub;
        Num<R>::uni2(st.next(), ua, ub);
        const R a = R(2) * ua - R(1);
        const R b = R(2) * ub - R(1);
        const R q = a * a + b * b;
        if (q > R(0) && q < R(1)) {
            const R f = Num<R>::sqrt(Num<R>::div(R(-2) * Num<R>::log(q), q));
            n0 = (a * f) * sd;
            n1 = (b * f) * sd;
            return;
        }
    }
}

// One polar-method attempt on two FP32 uniforms; true when accepted.
__device__ __forceinline__ bool polar_try(uint32_t wa, uint32_t wb, float sd, float& n0, float& n1) {
    const float a = 2.0f * u24(wa) - 1.0f, b = 2.0f * u24(wb) - 1.0f;
    const float q = a * a + b * b;
    if (!(q > 0.0f && q < 1.0f)) return false;
    const float f = Num<float>::sqrt(Num<float>::div(-2.0f * Num<float>::log(q), q));
    n0 = (a * f) * sd;
    n1 = (b * f) * sd;
    return true;
}

// The fast mode uses all four words of a call: two polar attempts per call.
template <>
__device__ __forceinline__ void normal_pair<float>(Stream& st, float sd, float& n0, float& n1) {
    for (;;) {
        const uint4 x = st.next();
        if (polar_try(x.x, x.y, sd, n0, n1) || polar_try(x.z, x.w, sd, n0, n1)) return;
    }
}

// The draws of one re-emission from a plate at T = sd^2: the normal speed
// sqrt(-2 T ln U) and a tangential pair.  FP64: call 0 gives U, the pair
// follows from later calls (the recipe's order).  FP32: call 0 gives U (word 0)
// and the first polar attempt (words 1 and 2).
template <class R>
__device__ __forceinline__ void wall_draws(Stream& st, R sd, R& vn, R& t0, R& t1) {
    R ua, ub;
    Num<R>::uni2(st.next(), ua, ub);
    vn = Num<R>::sqrt(R(-2) * Num<R>::log(ua)) * sd;
    normal_pair<R>(st, sd, t0, t1);
}

template <>
__device__ __forceinline__ void wall_draws<float>(Stream& st, float sd, float& vn, float& t0, float& t1) {
    const uint4 x = st.next();
    vn = Num<float>::sqrt(-2.0f * Num<float>::log(u24(x.x))) * sd;
    if (!polar_try(x.y, x.z, sd, t0, t1)) normal_pair<float>(st, sd, t0, t1);
}

// The normal speed of a re-emission alone, from the same words and in the
// same arithmetic as wall_draws (it never depends on the tangential pair):
// what a flight of the position alone needs.
template <class R>
__device__ __forceinline__ R wall_normal_speed(Stream& st, R sd) {
    R ua, ub;
    Num<R>::uni2(st.next(), ua, ub);
    return Num<R>::sqrt(R(-2) * Num<R>::log(ua)) * sd;
}

template <>
__device__ __forceinline__ float wall_normal_speed<float>(Stream& st, float sd) {
    const uint4 x = st.next();
    return Num<float>::sqrt(-2.0f * Num<float>::log(u24(x.x))) * sd;
}

// Marsaglia (1972): uniform point on the unit sphere from a point uniform in
// the unit disc: (2a sqrt(1-q), 2b sqrt(1-q), 1 - 2q).
template <class R>
__device__ __forceinline__ void sphere_point(Stream& st, R& dx, R& dy, R& dz) {
#pragma clang fp contract(off)
    for (;;) {
        R ua, ub;
        Num<R>::uni2(st.next(), ua, ub);
        const R a = R(2) * ua - R(1);
        const R b = R(2) * ub - R(1);
        const R q = a * a + b * b;
        if (q < R(1)) {
            const R r = R(2) * Num<R>::sqrt(R(1) - q);
            dx = a * r;
            dy = b * r;
            dz = R(1) - R(2) * q;
            return;
        }
    }
}

}  // namespace dsmc
