// pic_device.h -- device-side building blocks of the gfx950 PIC step.
//
// Everything here is templated on the storage/compute type T (float or
// double).  Particles are an int32 cell (packed radial and meridional index)
// plus an in-cell offset in [0, 1); the push works with local increments so
// that an FP32 offset keeps ~1e-7 cell resolution at any radius.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kCellOff = 0x4000;            // radial index bias inside a packed cell
constexpr uint32_t kDead = 0xFFFFFFFFu;     // packed cell of a deleted particle
constexpr double kPi = 3.14159265358979323846;

__host__ __device__ inline uint32_t pack_cell(int i, int j)
{
    return ((uint32_t)(i + kCellOff) << 16) | (uint32_t)j;
}
__host__ __device__ inline int cell_i(uint32_t c) { return (int)(c >> 16) - kCellOff; }
__host__ __device__ inline int cell_j(uint32_t c) { return (int)(c & 0xFFFFu); }

// Field storage: every component (E_r, E_th, E_ph, B_r, B_th, B_ph and the
// face charges F_r, F_th, F_ph) uses one padded layout, element (i, j) at
// (i + G) * pitch + j, rows i = -G .. nr + G, columns j = 0 .. nth.  Ghost
// rows of E and B stay zero: the plasma field vanishes in the conductors.
struct Layout {
    int nr, nth, G, pitch;
    __host__ __device__ int rows() const { return nr + 1 + 2 * G; }
    __host__ __device__ size_t at(int i, int j) const { return (size_t)(i + G) * pitch + j; }
    __host__ __device__ size_t size() const { return (size_t)rows() * pitch; }
};

enum : int { cER = 0, cETH = 1, cEPH = 2, cBR = 3, cBTH = 4, cBPH = 5, cFR = 6, cFTH = 7, cFPH = 8 };

template <typename T>
struct Fields {
    T *c[9];
};

// Pointers into device memory.  Pointers that kernels read from a table in
// memory are generic to the compiler, which then emits FLAT instructions
// (slower waits, no scalar base); cast to the global address space they
// give global_* loads, stores and atomics.
template <typename U>
using gptr = __attribute__((address_space(1))) U *;
template <typename U>
__device__ __forceinline__ gptr<U> glb(U *p)
{
    return (gptr<U>)p;
}
template <typename U>
__device__ __forceinline__ void atomic_add(gptr<U> p, U v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U>
__device__ __forceinline__ U atomic_add_fetch_old(gptr<U> p, U v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or(gptr<int> p, int v)
{
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
struct GFields {
    gptr<T> c[9];
};

// ---------------------------------------------------------------------
// Math policy.  FP32: hardware reciprocal, reciprocal square root and
// square root (1 ulp), exp via v_exp_f32, and short series for the small
// arguments the push sees (log1p of r'/r - 1, atan of the azimuthal step),
// falling back to the library outside their range; all far inside the FP32
// parity tolerance.  FP64: the hardware reciprocal estimates refined by
// Newton steps, IEEE square root where the argument can be zero, and series
// of the same kind with more terms (exp, log1p, atan), each within an ulp of
// the exact value, so that parity with the FP64 oracle holds at 1e-12.
// ---------------------------------------------------------------------
template <typename T>
struct FM;

template <>
struct FM<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float sqrt_pos(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // sqrt(x) and 1/sqrt(x) of x > 0 from one hardware reciprocal square root
    static __device__ __forceinline__ void sqrt_rsqrt(float x, float &s, float &is)
    {
        is = __builtin_amdgcn_rsqf(x);
        s = x * is;
    }
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
    // log(1 + e): alternating series through e^6 for |e| < 1/32 (truncation
    // below e^7 / 7 < 2^-33 |e|, under FP32 rounding)
    static __device__ __forceinline__ float log1p(float e)
    {
        if (fabsf(e) < 0.03125f) {
            float v = 0.2f - e * (1.0f / 6);
            v = 0.25f - e * v;
            v = 1.0f / 3 - e * v;
            v = 0.5f - e * v;
            return e - e * e * v;
        }
        return log1pf(e);
    }
    // atan2(y, x) for x > 0 and |y| < x / 4: odd series of atan(y / x)
    // through t^13 (truncation < t^15 / 15 < 1e-10), else the library
    static __device__ __forceinline__ float atan2(float y, float x)
    {
        if (x > 0.f && fabsf(y) < 0.25f * x) {
            const float t = y * __builtin_amdgcn_rcpf(x), t2 = t * t;
            float v = 1.0f / 11 - t2 * (1.0f / 13);
            v = 1.0f / 9 - t2 * v;
            v = 1.0f / 7 - t2 * v;
            v = 0.2f - t2 * v;
            v = 1.0f / 3 - t2 * v;
            return t - t * t2 * v;
        }
        return atan2f(y, x);
    }
};

template <>
struct FM<double> {
    // 1/x and 1/sqrt(x) of normal x > 0 from the hardware estimates (good to
    // about 2^-23) and two Newton steps, each of which squares the relative
    // error: within an ulp of the rounded result, in a third of the
    // instructions of IEEE division and square root
    static __device__ __forceinline__ double rcp(double x)
    {
        double y = __builtin_amdgcn_rcp(x);
        y = fma(y, fma(-x, y, 1.0), y);
        return fma(y, fma(-x, y, 1.0), y);
    }
    static __device__ __forceinline__ double rsqrt(double x)
    {
        double y = __builtin_amdgcn_rsq(x);
        y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
        return fma(0.5 * y, fma(-(x * y), y, 1.0), y);
    }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); } // x = 0 occurs (the poles)
    static __device__ __forceinline__ double div(double a, double b) { return a * rcp(b); }
    // sqrt(x) of normal x > 0: x / sqrt(x) with one correction from its residual
    static __device__ __forceinline__ double sqrt_pos(double x)
    {
        const double is = rsqrt(x), s0 = x * is;
        return fma(fma(-s0, s0, x), 0.5 * is, s0);
    }
    // sqrt(x) and 1/sqrt(x) of normal x > 0; the square root takes one
    // correction from its residual
    static __device__ __forceinline__ void sqrt_rsqrt(double x, double &s, double &is)
    {
        is = rsqrt(x);
        const double s0 = x * is;
        s = fma(fma(-s0, s0, x), 0.5 * is, s0);
    }
    // exp(x): Taylor series through x^8 for |x| < 1/32 (truncation below
    // x^9 / 9! < 2^-63), else the library
    static __device__ __forceinline__ double exp(double x)
    {
        if (fabs(x) < 0.03125) {
            double v = fma(x, 1.0 / 40320, 1.0 / 5040); // 1/8!, 1/7!
            v = fma(x, v, 1.0 / 720);
            v = fma(x, v, 1.0 / 120);
            v = fma(x, v, 1.0 / 24);
            v = fma(x, v, 1.0 / 6);
            v = fma(x, v, 0.5);
            v = fma(x, v, 1.0);
            return fma(x, v, 1.0);
        }
        return ::exp(x);
    }
    // log(1 + e): alternating series through e^12 for |e| < 1/32 (truncation
    // below e^13 / 13 < 2^-63 |e|, under FP64 rounding), else the library
    static __device__ __forceinline__ double log1p(double e)
    {
        if (fabs(e) < 0.03125) {
            double v = 1.0 / 12;
#pragma unroll
            for (int k = 11; k >= 2; --k) v = 1.0 / k - e * v;
            return e - e * e * v;
        }
        return ::log1p(e);
    }
    // atan2(y, x) for x > 0 and |y| < x / 8: odd series of atan(y / x)
    // through t^17 (truncation < t^19 / 19 < 2^-58 |t|), else the library
    static __device__ __forceinline__ double atan2(double y, double x)
    {
        if (x > 0.0 && fabs(y) < 0.125 * x) {
            const double t = div(y, x), t2 = t * t;
            double v = 1.0 / 17;
#pragma unroll
            for (int m = 7; m >= 1; --m) v = 1.0 / (2 * m + 1) - t2 * v;
            return t - t * t2 * v;
        }
        return ::atan2(y, x);
    }
};

// Analytic initial ("vacuum") field of the rotating conductor, Sec. 5.2 and
// Sec. 4.3; local (r, theta, phi) components at radius r, cos/sin theta.
struct Background {
    int kind;          // PIC_BG_*
    double B0, r0;     // surface field and conductor radius
};

// The increments are formed in scalars and added once at the end, so that
// the compiler keeps E and B in registers whatever the case.
template <typename T>
__device__ inline void add_background(const Background &bg, T inv_rl, bool inside, T r, T ir, T k, T s, T E[3],
                                      T B[3])
{
    const T B0 = (T)bg.B0, r0 = (T)bg.r0;
    T e0 = (T)0, e1 = (T)0, b0 = (T)0, b1 = (T)0;
    switch (bg.kind) {
    case 1: // uniform B along the axis
        b0 = B0 * k;
        b1 = -(B0 * s);
        break;
    case 2: { // monopole: inside corotation, outside the vacuum l = 1 field
        const T q = r0 * ir;
        b0 = B0 * q * q;
        if (inside) {
            e1 = -(B0 * r0 * q * s * inv_rl);
        } else {
            const T a = B0 * r0 * q * q * q * inv_rl;
            e0 = -((T)2 * a * k);
            e1 = -(a * s);
        }
        break;
    }
    case 3:
    case 4: { // dipole; corotation inside (or everywhere for the drift test), l = 2 vacuum outside
        const T q = r0 * ir;
        const T q3 = q * q * q;
        b0 = (T)2 * B0 * q3 * k;
        b1 = B0 * q3 * s;
        if (inside || bg.kind == 4) {
            const T a = B0 * r0 * q * q * inv_rl;
            e0 = a * s * s;
            e1 = -((T)2 * a * s * k);
        } else {
            const T a = (T)2 * B0 * r0 * q3 * q * inv_rl;
            e0 = -(a * (T)0.5 * ((T)3 * k * k - (T)1));
            e1 = -(a * s * k);
        }
        break;
    }
    default:
        break;
    }
    E[0] += e0;
    E[1] += e1;
    B[0] += b0;
    B[1] += b1;
}

template <typename T>
__device__ inline void add_background(const Background &bg, T inv_rl, bool inside, T r, T k, T s, T E[3], T B[3])
{
    add_background(bg, inv_rl, inside, r, FM<T>::rcp(r), k, s, E, B);
}

// ---------------------------------------------------------------------
// Movers (Cartesian).  u = gamma v / c, eps = q dt / (2 m c).
// ---------------------------------------------------------------------

// Returns 1 / gamma of the new momentum.
template <typename T>
__device__ inline T vay_push(T u[3], const T E[3], const T B[3], T eps)
{
    const T ig = FM<T>::rsqrt((T)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const T vx = u[0] * ig, vy = u[1] * ig, vz = u[2] * ig;
    // half electric kick twice and the magnetic rotation with the old velocity
    const T px = u[0] + (T)2 * eps * E[0] + eps * (vy * B[2] - vz * B[1]);
    const T py = u[1] + (T)2 * eps * E[1] + eps * (vz * B[0] - vx * B[2]);
    const T pz = u[2] + (T)2 * eps * E[2] + eps * (vx * B[1] - vy * B[0]);
    const T tx = eps * B[0], ty = eps * B[1], tz = eps * B[2];
    const T tau2 = tx * tx + ty * ty + tz * tz;
    const T us = px * tx + py * ty + pz * tz;
    const T sg = (T)1 + px * px + py * py + pz * pz - tau2;
    const T g2 = (T)0.5 * (sg + FM<T>::sqrt_pos(sg * sg + (T)4 * (tau2 + us * us))); // > 0: sg >= 1 where tau = 0
    const T ign = FM<T>::rsqrt(g2);
    const T ax = tx * ign, ay = ty * ign, az = tz * ign;
    const T sf = FM<T>::rcp((T)1 + ax * ax + ay * ay + az * az);
    const T pt = px * ax + py * ay + pz * az;
    u[0] = sf * (px + pt * ax + (py * az - pz * ay));
    u[1] = sf * (py + pt * ay + (pz * ax - px * az));
    u[2] = sf * (pz + pt * az + (px * ay - py * ax));
    return ign;
}

template <typename T>
__device__ inline void boris_push(T u[3], const T E[3], const T B[3], T eps)
{
    const T mx = u[0] + eps * E[0], my = u[1] + eps * E[1], mz = u[2] + eps * E[2];
    const T ig = FM<T>::rsqrt((T)1 + mx * mx + my * my + mz * mz);
    const T tx = eps * B[0] * ig, ty = eps * B[1] * ig, tz = eps * B[2] * ig;
    const T f = (T)2 * FM<T>::rcp((T)1 + tx * tx + ty * ty + tz * tz);
    const T qx = mx + (my * tz - mz * ty), qy = my + (mz * tx - mx * tz), qz = mz + (mx * ty - my * tx);
    u[0] = mx + f * (qy * tz - qz * ty) + eps * E[0];
    u[1] = my + f * (qz * tx - qx * tz) + eps * E[1];
    u[2] = mz + f * (qx * ty - qy * tx) + eps * E[2];
}

// ---------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), used for the
// positions of injected pairs.
// ---------------------------------------------------------------------
__device__ inline void philox4x64(uint64_t x[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t lo0 = M0 * x[0], hi0 = __umul64hi(M0, x[0]);
        const uint64_t lo1 = M1 * x[2], hi1 = __umul64hi(M1, x[2]);
        const uint64_t n0 = hi1 ^ x[1] ^ k0, n2 = hi0 ^ x[3] ^ k1;
        x[0] = n0;
        x[1] = lo1;
        x[2] = n2;
        x[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

} // namespace pic
