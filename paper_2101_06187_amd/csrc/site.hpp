// Per-site device building blocks of the RLBM step: storage forms, pull
// streaming, moments, the FP64 Landau-frame solve and the collision/force
// update.  Shared by the step kernel and the auxiliary kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "engine.hpp"

// Only the fma() calls written out below fuse a multiply and an add: the
// compiler does not contract other a * b + c on its own.  Every kernel form
// inlines the same per-site code into different surroundings, and this keeps
// their results bitwise identical.
#pragma clang fp contract(off)

namespace rlbm {

// ---------------------------------------------------------------------------
// compile-time loop
// ---------------------------------------------------------------------------
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// global address space and wave-uniform values.  Casting a uniform base to the
// global address space lets the compiler address population planes as
// (scalar 64-bit base) + (32-bit per-lane offset).
// ---------------------------------------------------------------------------
template <class X>
using gp = __attribute__((address_space(1))) X*;
// Constant address space: memory that no wave of the running kernel writes.
// A wave-uniform address into it is read with scalar loads into SGPRs.
template <class X>
using kp = __attribute__((address_space(4))) X*;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (long long)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint64_t uni(uint64_t v) { return (uint64_t)uni((long long)v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
    return __longlong_as_double(uni(__double_as_longlong(v)));
}
template <class P>
__device__ __forceinline__ P* uni(P* p) {
    return (P*)uni((long long)(uintptr_t)p);
}

// ---------------------------------------------------------------------------
// storage forms.  Registers hold f' = F - shift; memory holds raw(f').
// ---------------------------------------------------------------------------
// FP32 -> BF16, round to nearest even: gfx950's v_cvt_pk_bf16_f32 (one
// instruction; NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

struct StF64 {
    using raw = double;
    using T = double;
    static constexpr int shift = 0;
    static constexpr int id = RLBM_F64;
    template <class P> __device__ static T ld(P p) { return *p; }
    template <class P> __device__ static void st(P p, T v) { *p = v; }
    template <class P> __device__ static void st_nt(P p, T v) { __builtin_nontemporal_store(v, p); }
    __device__ static raw fma_round(T a, T b, T c) { return fma(a, b, c); }
    __device__ static double to64(raw v) { return v; }
    __device__ static raw from64(double v) { return v; }
};
struct StF32 {            // stores F - 1 in FP32: the deviation keeps all 24 bits
    using raw = float;
    using T = float;
    static constexpr int shift = 1;
    static constexpr int id = RLBM_F32;
    template <class P> __device__ static T ld(P p) { return *p; }
    template <class P> __device__ static void st(P p, T v) { *p = v; }
    template <class P> __device__ static void st_nt(P p, T v) { __builtin_nontemporal_store(v, p); }
    __device__ static raw fma_round(T a, T b, T c) { return fmaf(a, b, c); }
    __device__ static double to64(raw v) { return (double)v; }
    __device__ static raw from64(double v) { return (float)v; }
};
struct StF16S {
    using raw = _Float16;
    using T = float;
    static constexpr int shift = 1;
    static constexpr int id = RLBM_F16S;
    template <class P> __device__ static T ld(P p) { return (float)*p; }
    template <class P> __device__ static void st(P p, T v) { *p = (_Float16)v; }
    __device__ static T from_bits(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
    template <class P> __device__ static void st_nt(P p, T v) { __builtin_nontemporal_store((_Float16)v, p); }
    // a * b + c rounded once, from its exact value, to FP16 (round to nearest
    // even): v_fma_mixlo_f16 with three FP32 operands.  Written out so that
    // every kernel form rounds the same way: left to itself the compiler fuses
    // the FP32 multiply-add and the conversion in some kernels and rounds
    // twice (FP32, then FP16, packing two results) in others.
    __device__ static raw fma_round(T a, T b, T c) {
        uint32_t r;   // the instruction writes the low half
        asm("v_fma_mixlo_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
        return __builtin_bit_cast(_Float16, (uint16_t)r);
    }
    __device__ static double to64(raw v) { return (double)(float)v; }
    __device__ static raw from64(double v) { return (_Float16)(float)v; }
    // Two adjacent columns in one 32-bit word, the even one in the low half.
    // pk_first rounds a * b + c into the low half (the high half is left
    // undefined); pk_second rounds the next column's into the high half of
    // that word and keeps its low half (v_fma_mixhi_f16: the same single
    // rounding as fma_round, written to the other half).
    using pair_tmp = uint32_t;
    __device__ static pair_tmp pk_first(T a, T b, T c) {
        uint32_t r;
        asm("v_fma_mixlo_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
        return r;
    }
    __device__ static uint32_t pk_second(pair_tmp w, T a, T b, T c) {
        asm("v_fma_mixhi_f16 %0, %1, %2, %3" : "+v"(w) : "v"(a), "v"(b), "v"(c));
        return w;
    }
    __device__ static T lo(uint32_t u) { return from_bits((uint16_t)(u & 0xffffu)); }
    __device__ static T hi(uint32_t u) { return from_bits((uint16_t)(u >> 16)); }
};
struct StBF16S {
    using raw = uint16_t;
    using T = float;
    static constexpr int shift = 1;
    static constexpr int id = RLBM_BF16S;
    template <class P> __device__ static T ld(P p) { return __uint_as_float((uint32_t)*p << 16); }
    template <class P> __device__ static void st(P p, T v) { *p = f32_to_bf16_rne(v); }
    __device__ static T from_bits(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
    // the FP32 multiply-add, rounded to nearest even BF16
    __device__ static raw fma_round(T a, T b, T c) { return f32_to_bf16_rne(fmaf(a, b, c)); }
    template <class P> __device__ static void st_nt(P p, T v) {
        __builtin_nontemporal_store(f32_to_bf16_rne(v), p);
    }
    __device__ static double to64(raw v) { return (double)__uint_as_float((uint32_t)v << 16); }
    __device__ static raw from64(double v) { return f32_to_bf16_rne((float)v); }
    // Two adjacent columns in one 32-bit word, the even one in the low half:
    // the first column's FP32 multiply-add is kept until the second's, then
    // both are rounded to nearest even BF16 by one v_cvt_pk_bf16_f32.
    using pair_tmp = float;
    __device__ static pair_tmp pk_first(T a, T b, T c) { return fmaf(a, b, c); }
    __device__ static uint32_t pk_second(pair_tmp w, T a, T b, T c) {
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        const f32x2 v = {w, fmaf(a, b, c)};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    }
    __device__ static T lo(uint32_t u) { return __uint_as_float(u << 16); }
    __device__ static T hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
};

// ---------------------------------------------------------------------------
// pull streaming by linear interpolation (Sec. III B), periodic lattice.
// Populations are stored in row bricks (pop_index): population q of a site is
// q * 64 elements after population 0 of the same site.
// rows[j] is the (wave-uniform) address of lattice row y + j - 1, cols[i] the
// per-lane byte offset (col_bytes) of column x + i - 1.
// The population of direction c arriving at x comes from x - cfl * v: for
// c_x > 0 it lies between x - 1 (weight a) and x (weight 1 - a), a = cfl |v_x|;
// for c_x, c_y both non-zero (|v_x| = |v_y|) the bilinear weights are
// (1 - a)^2 (own node), a (1 - a) (each edge neighbour), a^2 (diagonal).
// ---------------------------------------------------------------------------
// Interpolation formulas.  MIX (16-bit storage): the node values enter fused
// multiply-adds, which take a 16-bit operand as it is (v_fma_mix_f32), rather
// than sums or differences, which need each value converted first (only the
// own node of the bilinear sum enters a product).  Otherwise (FP32, FP64
// storage) the sums of node values are formed first.  Every kernel form uses
// the same formula for a storage type, so the forms agree bit for bit.
template <class S>
constexpr bool mix_interp = sizeof(typename S::raw) == 2;

// (1 - t) p + t q
template <bool MIX, class T>
__device__ __forceinline__ T lerp(T p, T q, T t) {
    if constexpr (MIX) return fma(t, q, fma(-t, p, p));
    else return fma(t, q - p, p);
}

template <class T>
struct InterpW {
    T a[3];       // cfl |v| for 1, 2, 3 non-zero cube components
    T w00[3], w10[3], w11[3];
    __device__ void set(T a1, T a2, T a3) {
        a[0] = a1; a[1] = a2; a[2] = a3;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T b = (T)1 - a[i];
            w00[i] = b * b;
            w10[i] = a[i] * b;
            w11[i] = a[i] * a[i];
        }
    }
};

// Bilinear interpolation with weights of W for i + 1 non-zero components:
// o own node, h its upstream neighbour in the row, v in the column, dg the
// diagonal one.
template <bool MIX, class T>
__device__ __forceinline__ T bilerp(T o, T h, T v, T dg, const InterpW<T>& W, int i) {
    if constexpr (MIX) return fma(W.w11[i], dg, fma(W.w10[i], h, fma(W.w10[i], v, W.w00[i] * o)));
    else return fma(W.w11[i], dg, fma(W.w10[i], h + v, W.w00[i] * o));
}

// The interpolation itself, for any source of the 3 x 3 neighbourhood:
// ld(q, j, i) returns population q at row y + j - 1, column x + i - 1.
template <class St, int SM, bool MIX, class T, class Ld>
__device__ __forceinline__ void stream_interp(Ld&& ld, const InterpW<T>& W, T (&f)[St::Q]) {
    constexpr bool UNIT = SM == kStreamUnit;
    sfor<0, St::Q>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        constexpr Dir d = St::dir[q];
        constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
        constexpr int ux = d.cx > 0 ? 0 : (d.cx < 0 ? 2 : 1);   // upstream column index
        constexpr int uy = d.cy > 0 ? 0 : (d.cy < 0 ? 2 : 1);   // upstream row index
        auto L = [&](int j, int i) -> T { return ld(q, j, i); };
        if constexpr (d.cx == 0 && d.cy == 0) {
            f[q] = L(1, 1);
        } else if constexpr (d.cy == 0) {
            if constexpr (UNIT && n == 1) f[q] = L(1, ux);
            else f[q] = lerp<MIX>(L(1, 1), L(1, ux), W.a[n - 1]);
        } else if constexpr (d.cx == 0) {
            if constexpr (UNIT && n == 1) f[q] = L(uy, 1);
            else f[q] = lerp<MIX>(L(1, 1), L(uy, 1), W.a[n - 1]);
        } else {
            const T h = L(1, ux), v = L(uy, 1);
            const T dg = L(uy, ux);
            f[q] = bilerp<MIX>(L(1, 1), h, v, dg, W, n - 1);
        }
    });
}

// from global memory: rows[j] row y + j - 1 (wave-uniform), cols[i] the
// per-lane byte offset of column x + i - 1
template <class S, class St, int SM, class T>
__device__ __forceinline__ void stream_pull(const char* const (&rows)[3],
                                            const uint32_t (&cols)[3], const InterpW<T>& W,
                                            T (&f)[St::Q]) {
    using raw = typename S::raw;
    constexpr long long plane_bytes = kTileW * sizeof(raw);
    stream_interp<St, SM, mix_interp<S>>(
        [&](int q, int j, int i) -> T {
            return (T)S::ld((gp<const raw>)(rows[j] + (long long)q * plane_bytes + cols[i]));
        },
        W, f);
}

// ---------------------------------------------------------------------------
// 1 < cfl <= 2.  A population with displacement a = cfl |v_x| along x comes
// from between the nodes floor(a) and floor(a) + 1 upstream; with the 1-D
// weights of the upstream offsets 0, 1, 2
//   a <= 1: (1 - a, a, 0),   1 < a <= 2: (0, 2 - a, a - 1),
// the interpolant is sum_k c_k F(x - k sign(c_x)), and for c_x, c_y both
// non-zero (|v_x| = |v_y|) the tensor product sum_{i,j} c_i c_j F(x - i, y - j).
// rows[j] is the row y + j - 2, cols[i] the column x + i - 2.
// ---------------------------------------------------------------------------
template <class T>
struct InterpW2 {
    T c[3][3];    // [n - 1][offset]: 1-D weights for 1, 2, 3 non-zero components
    __device__ void set(T a1, T a2, T a3) {
        const T a[3] = {a1, a2, a3};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool far = a[i] > (T)1;
            c[i][0] = far ? (T)0 : (T)1 - a[i];
            c[i][1] = far ? (T)2 - a[i] : a[i];
            c[i][2] = far ? a[i] - (T)1 : (T)0;
        }
    }
};

template <class S, class St, class T>
__device__ __forceinline__ void stream_pull_h2(const char* const (&rows)[5],
                                               const uint32_t (&cols)[5], const InterpW2<T>& W,
                                               T (&f)[St::Q]) {
    using raw = typename S::raw;
    constexpr long long plane_bytes = kTileW * sizeof(raw);
    sfor<0, St::Q>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        constexpr Dir d = St::dir[q];
        constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
        constexpr int sx = d.cx > 0 ? -1 : (d.cx < 0 ? 1 : 0);   // column step upstream
        constexpr int sy = d.cy > 0 ? -1 : (d.cy < 0 ? 1 : 0);   // row step upstream
        auto L = [&](int j, int i) -> T {                        // j rows, i columns upstream
            return (T)S::ld((gp<const raw>)(rows[2 + sy * j] + (long long)q * plane_bytes +
                                            cols[2 + sx * i]));
        };
        const T* c = W.c[n > 0 ? n - 1 : 0];
        if constexpr (d.cx == 0 && d.cy == 0) {
            f[q] = L(0, 0);
        } else if constexpr (d.cy == 0) {
            f[q] = fma(c[2], L(0, 2), fma(c[1], L(0, 1), c[0] * L(0, 0)));
        } else if constexpr (d.cx == 0) {
            f[q] = fma(c[2], L(2, 0), fma(c[1], L(1, 0), c[0] * L(0, 0)));
        } else {
            T acc = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const T r = fma(c[2], L(j, 2), fma(c[1], L(j, 1), c[0] * L(j, 0)));
                acc = fma(c[j], r, acc);
            }
            f[q] = acc;
        }
    });
}

// ---------------------------------------------------------------------------
// moments (Sec. III A): E = sum w F, J = sum w F v, Pi = sum w F v v and, for
// the force, R = sum w F v v v (in-plane components), from shifted registers.
// Pair sums S = F(+u) + F(-u) carry the even moments, D = F(+u) - F(-u) the
// odd ones.
// ---------------------------------------------------------------------------
template <class T>
struct Moments {
    T E, Jx, Jy, Pxx, Pxy, Pyy, Rxxx, Rxxy, Rxyy, Ryyy;
};

template <class St, bool WITH_R, class T>
__device__ __forceinline__ Moments<T> moments(const T (&f)[St::Q]) {
    Moments<T> m{};
    sfor<0, St::NC>([&](auto ic) {
        constexpr DirClass C = St::cls[ic];
        constexpr double um = comp_mag(C.ncomp);
        constexpr double ux = C.sx * um, uy = C.sy * um;
        T Sp = f[C.first];
        sfor<1, C.nplus>([&](auto i) { Sp += f[C.first + decltype(i)::value]; });
        T S = Sp, Dd = Sp;
        if constexpr (C.nminus > 0) {
            T Sm = f[C.first + C.nplus];
            sfor<1, C.nminus>([&](auto i) { Sm += f[C.first + C.nplus + decltype(i)::value]; });
            S = Sp + Sm;
            Dd = Sp - Sm;
        }
        m.E = fma((T)C.w, S, m.E);
        if constexpr (ux != 0.0) {
            m.Pxx = fma((T)(C.w * ux * ux), S, m.Pxx);
            m.Jx = fma((T)(C.w * ux), Dd, m.Jx);
        }
        if constexpr (uy != 0.0) {
            m.Pyy = fma((T)(C.w * uy * uy), S, m.Pyy);
            m.Jy = fma((T)(C.w * uy), Dd, m.Jy);
        }
        if constexpr (ux != 0.0 && uy != 0.0) m.Pxy = fma((T)(C.w * ux * uy), S, m.Pxy);
        if constexpr (WITH_R) {
            if constexpr (ux != 0.0) m.Rxxx = fma((T)(C.w * ux * ux * ux), Dd, m.Rxxx);
            if constexpr (ux != 0.0 && uy != 0.0) {
                m.Rxxy = fma((T)(C.w * ux * ux * uy), Dd, m.Rxxy);
                m.Rxyy = fma((T)(C.w * ux * uy * uy), Dd, m.Rxyy);
            }
            if constexpr (uy != 0.0) m.Ryyy = fma((T)(C.w * uy * uy * uy), Dd, m.Ryyy);
        }
    });
    return m;
}

// ---------------------------------------------------------------------------
// FP64 helpers: reciprocal and reciprocal square root from the hardware
// estimates refined by Newton steps (each step doubles the correct bits).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// ---------------------------------------------------------------------------
// Landau frame (Sec. III A/B).  For a state without out-of-plane momentum the
// condition T^{mu nu} u_nu = -eps u^mu reduces to
//     (eps I + Pi) beta = J,   eps = E - J . beta,
// i.e. eps is the root of g(eps) = eps - E + J^T (eps I + Pi)^-1 J with
// g'(eps) = 1 - |beta|^2 > 0.  Newton's method from the small-velocity
// estimate eps0 = E - |J|^2 D / ((D+1) E).  Since 0 < g'' <= 2 |J|^2 / eps^3
// and |J| <= (4/3) eps gamma^2 |beta|, a correction |de| <= 2e-8 eps leaves an
// error below (16/9) gamma^4 beta^2 / (1 - beta^2) * 4e-16 eps (under 5e-16 eps
// for |beta| <= 1/2): the iteration then only solves for beta at the new eps.
// Returns false if it does not converge or the result is unphysical.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ bool landau64(double E, double Jx, double Jy, double Pxx,
                                         double Pxy, double Pyy, double& eps, double& bx,
                                         double& by) {
    const double J2 = fma(Jx, Jx, Jy * Jy);
    const double Pxy2 = Pxy * Pxy;
    double e = fma(-J2 * ((double)D / (D + 1)), rcp64(E), E);
    bool ok = false;
    auto solve_beta = [&](double ee) {
        const double a = ee + Pxx, c = ee + Pyy;
        const double inv = rcp64(fma(a, c, -Pxy2));
        bx = fma(c, Jx, -Pxy * Jy) * inv;
        by = fma(a, Jy, -Pxy * Jx) * inv;
    };
    for (int it = 0; it < 16; ++it) {
        solve_beta(e);
        const double g = fma(Jx, bx, fma(Jy, by, e - E));
        const double de = g * rcp64(fma(-bx, bx, fma(-by, by, 1.0)));
        e -= de;
        // converged: beta of this pass belongs to eps to within |de| ~ 1 ulp
        if (!(fabs(de) > 4e-16 * fabs(e))) { ok = true; break; }
        if (fabs(de) <= 2e-8 * fabs(e)) {
            solve_beta(e);
            ok = true;
            break;
        }
    }
    eps = e;
    const double b2 = fma(bx, bx, by * by);
    return ok && e > 0.0 && b2 < 1.0 && isfinite(e) && isfinite(b2);
}

// Equilibrium coefficients (Sec. III B, second-order projection of the
// Juettner distribution): F_eq(v) = A0 + B t + C t^2 with t = beta . v,
//   T00 = (eps + P) gamma^2 - P,  P = eps / D,
//   B = D (eps + P) gamma^2,  C = D (D+2)/2 (eps + P) gamma^2,
//   A0 = T00 - C beta^2 / D.
template <int D>
__device__ __forceinline__ void eq_coeffs(double eps, double bx, double by, double& A0,
                                          double& B, double& C, double& gamma) {
    const double b2 = fma(bx, bx, by * by);
    gamma = rsqrt64(1.0 - b2);
    const double g2 = gamma * gamma;
    constexpr double invD = 1.0 / D;
    const double hp = eps * ((D + 1.0) / D) * g2;     // (eps + P) gamma^2
    B = D * hp;
    C = (D * (D + 2) * 0.5) * hp;
    A0 = fma(-C * b2, invD, fma(-eps, invD, hp));
}


// ---------------------------------------------------------------------------
// The per-site part of the step after streaming (Sec. III C (c)-(e)): moments,
// FP64 Landau frame, equilibrium coefficients, force field and projected force
// term, Anderson-Witting collision, store of the new populations of this site
// into the destination row drow at byte offset own.  f holds the streamed
// populations (minus the storage shift); (c1, s1) = (cos, sin)(2 pi x / nx).
// ---------------------------------------------------------------------------
template <class T>
struct SiteCtx {
    T ginv, dt;
    int K;                 // largest |kx| of the force table; -1 unforced
    const T* gtab;         // force table of this step
    int eta_s;             // 1: relaxation time tau(eps) = tau eps^(-1/4) (constant eta/s)
};

// ---------------------------------------------------------------------------
// Force field at a site, FP64 path: F_c(x, y) = sum_k cos(k a) P_c(k, y) -
// sin(k a) Q_c(k, y), a = 2 pi x / nx, from the FP64 force table
// [ny][K+1][4] = (Px, Qx, Py, Qy), cos/sin(k a) by the Chebyshev recurrence
// from (c1, s1) = (cos, sin)(a).  The table row of a wave's lattice row is the
// same for all its lanes and was written by an earlier launch (a launch only
// writes the tables of later steps), so it is read as constant memory: scalar
// loads, no VGPRs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void force_cheb64(const SiteCtx<double>& ctx, double c1, double s1,
                                             int y, double& Fx, double& Fy) {
    using T = double;
    const int K = ctx.K;
    Fx = 0;
    Fy = 0;
    if (K < 0) return;                  // this lattice is unforced
    const kp<const T> grow = (kp<const T>)ctx.gtab + (size_t)y * (K + 1) * 4;
    Fx = grow[0];
    Fy = grow[2];
    T cp = 1, sp = 0, ck = c1, sk = s1;
    const T two_c1 = c1 + c1;
    auto term = [&](T g0, T g1, T g2, T g3) {
        Fx = fma(ck, g0, fma(-sk, g1, Fx));
        Fy = fma(ck, g2, fma(-sk, g3, Fy));
        const T cn = fma(two_c1, ck, -cp);
        const T sn = fma(two_c1, sk, -sp);
        cp = ck; sp = sk; ck = cn; sk = sn;
    };
    // Batches of RB table rows: one round of scalar loads per batch.  Every
    // table buffer has kTableSlack values after its last row, so the last
    // batch may reach past row K; those values are never used.
    constexpr int RB = 4;
    static_assert(4 * (RB - 1) <= kTableSlack, "a batch may reach 4 RB - 4 values past row K");
    int k = 1;
    for (; k + RB - 1 <= K; k += RB) {
        T gv[4 * RB];
#pragma unroll
        for (int i = 0; i < 4 * RB; ++i) gv[i] = grow[4 * k + i];
#pragma unroll
        for (int i = 0; i < RB; ++i) term(gv[4 * i], gv[4 * i + 1], gv[4 * i + 2], gv[4 * i + 3]);
    }
    if (k <= K) {
        T gv[4 * RB];
#pragma unroll
        for (int i = 0; i < 4 * RB; ++i) gv[i] = grow[4 * k + i];
#pragma unroll
        for (int i = 0; i < RB; ++i)
            if (k + i <= K) term(gv[4 * i], gv[4 * i + 1], gv[4 * i + 2], gv[4 * i + 3]);
    }
}

// ---------------------------------------------------------------------------
// Force field, FP32 path: the same sum as a dot product of length J over the
// terms j = 2k (cos(k a), coefficient P_c(k, y)) and j = 2k + 1 (sin(k a),
// coefficient -Q_c(k, y)), J = 2 (K + 1) rounded up to 16 with zero terms.
// The basis cos/sin(k a) is a per-lattice table [nx][J] (FP32, rounded from
// FP64 values at the exactly reduced angles 2 pi (k x mod nx) / nx); the
// coefficients are the per-step table [ny][J / 16][16][2] (c = x, y).  The
// sums run over the jt = 2 (K + 1) terms that are not zero by construction.
// Four sums at once by v_mfma_f32_4x4x1_16b_f32: with the A operand of block
// ABID broadcast to all 16 blocks, lane 4 t + m supplies coefficient m of term
// 16 c + t and every lane its own basis value, and lane l accumulates
//   acc[m] = fma(C_m[j], B_j(x_l), acc[m])   for j = 0, 1, ..., jt - 1
// (each MFMA of K = 1 is one fused multiply-add per output, single rounding),
// i.e. the same FP32 chain in every kernel form.  The four outputs are two
// (Fx, Fy) pairs whose coefficients the lanes load: m = 0, 1 from one table
// row, m = 2, 3 from another (two rows, or two steps).
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kForceChunk = 16;       // basis terms per A-operand register

// 16 terms of chunk c: a = this lane's coefficient register, b = this lane's
// 16 basis values
__device__ __forceinline__ v4f force_chunk(v4f acc, float a, const v4f (&b)[4]) {
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[0][0], acc, 4, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[0][1], acc, 4, 1, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[0][2], acc, 4, 2, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[0][3], acc, 4, 3, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[1][0], acc, 4, 4, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[1][1], acc, 4, 5, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[1][2], acc, 4, 6, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[1][3], acc, 4, 7, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[2][0], acc, 4, 8, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[2][1], acc, 4, 9, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[2][2], acc, 4, 10, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[2][3], acc, 4, 11, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[3][0], acc, 4, 12, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[3][1], acc, 4, 13, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[3][2], acc, 4, 14, 0);
    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[3][3], acc, 4, 15, 0);
    return acc;
}

// The first n terms of a chunk only (1 <= n <= 16): the chunk holding the
// forcing's largest wave number ends with zero terms, which are skipped.
__device__ __forceinline__ v4f force_chunk_n(v4f acc, float a, const v4f (&b)[4], int n) {
    sfor<0, kForceChunk>([&](auto it) {
        constexpr int t = decltype(it)::value;
        if (t < n) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b[t / 4][t % 4], acc, 4, t, 0);
    });
    return acc;
}

// The same for two chains over one coefficient register: accA with the basis
// values bA, accB with bB (the two columns of a paired lane), interleaved so
// that each chain's next MFMA does not wait for its previous one; the first n
// terms of the chunk.
template <bool ALL>
__device__ __forceinline__ void force_chunk2(v4f& accA, v4f& accB, float a, const v4f (&bA)[4],
                                             const v4f (&bB)[4], int n = kForceChunk) {
    sfor<0, kForceChunk>([&](auto it) {
        constexpr int t = decltype(it)::value;
        if (ALL || t < n) {
            accA = __builtin_amdgcn_mfma_f32_4x4x1f32(a, bA[t / 4][t % 4], accA, 4, t, 0);
            accB = __builtin_amdgcn_mfma_f32_4x4x1f32(a, bB[t / 4][t % 4], accB, 4, t, 0);
        }
    });
}

// Terms in the last chunk of a sum over jt terms (1 .. 16).
__device__ __forceinline__ int force_tail(int jt) { return jt - kForceChunk * ((jt - 1) / kForceChunk); }

// Per-lane addressing of the coefficient loads: lane 4 t + m reads component
// m % 2 of term 16 c + t from row A (m < 2) or row B (m >= 2).
struct ForceLane {
    uint32_t off;         // 2 t + m % 2 (floats)
    bool hi;              // m >= 2
    __device__ void init(int lane) {
        off = (uint32_t)(2 * (lane >> 2) + (lane & 1));
        hi = (lane & 2) != 0;
    }
};

// The whole sum over the jt = 2 (K + 1) terms with the coefficient registers
// loaded here (one global load per chunk), for forms whose lanes read their
// basis from the global table: rowA / rowB point at the coefficient rows of
// the two output pairs, bas at this lane's basis row [J].
__device__ __forceinline__ v4f force_sum_global(const float* rowA, const float* rowB,
                                                const float* bas, int jt, const ForceLane& fl) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const gp<const float> row = (gp<const float>)(fl.hi ? rowB : rowA);
    const gp<const v4f> b4 = (gp<const v4f>)bas;
    const int nch = (jt + kForceChunk - 1) / kForceChunk;
    auto chunk = [&](int c, v4f (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = b4[4 * c + i];
        return row[32 * c + fl.off];
    };
    for (int c = 0; c + 1 < nch; ++c) {
        v4f b[4];
        const float a = chunk(c, b);
        acc = force_chunk(acc, a, b);
    }
    v4f b[4];
    const float a = chunk(nch - 1, b);
    return force_chunk_n(acc, a, b, force_tail(jt));
}

// fin(qc, a, b, c) receives population qc (a std::integral_constant) of the
// new state as the operands of the collision's last multiply-add:
// F_q - shift = a * b + c, to be rounded once to the storage type (as
// S::fma_round does).  (Fx, Fy) is the stirring force at the site (zero when
// unforced).
// A lane whose result is discarded passes live = false: it does not raise the
// stability flag.
template <class S, class St, bool FORCED, class T, class Fin>
__device__ __forceinline__ void update_site_fma(const T (&f)[St::Q], const SiteCtx<T>& ctx, T Fx,
                                                T Fy, Fin&& fin, int* d_flag, bool live = true) {
    constexpr int D = St::D;
    const T ginv = ctx.ginv, dt = ctx.dt;
    // (c) moments, Landau frame in FP64
    const Moments<T> m = moments<St, FORCED>(f);
    const double E64 = (double)m.E + (double)S::shift;
    const double dshift = (double)S::shift / D;     // sum_q w v_i v_i = 1/D per axis
    double eps, bx64, by64;
    const bool ok = landau64<D>(E64, (double)m.Jx, (double)m.Jy,
                                (double)m.Pxx + dshift, (double)m.Pxy,
                                (double)m.Pyy + dshift, eps, bx64, by64);
    if (!ok && live) *d_flag = 1;

    // (d) equilibrium F_eq - shift = A0' + B t + C t^2 (t = beta.v), and the
    // Anderson-Witting rate omega = g (1 - t), g = gamma / tau.  For the +v
    // and -v members of a class:
    //   omega (F_eq - shift) = E(t) +- O(t),
    //   E = g A0' + g (C - B) t^2,   O = g (B - A0') t - g C t^3.
    double A0d, Bd, Cd, gam;
    eq_coeffs<D>(eps, bx64, by64, A0d, Bd, Cd, gam);
    const double A0s = A0d - (double)S::shift;
    double g64 = gam * (double)ginv;
    // constant eta/s (Sec. III A): tau_R = 5 (eta/s) / T with T = eps^(1/4)
    // for massless particles at T0 = 1, so 1/tau scales as eps^(1/4)
    if (__builtin_expect(ctx.eta_s != 0, 0)) g64 *= rsqrt64(rsqrt64(eps));   // eps^(1/4)
    const T g = (T)g64;
    const T k0 = (T)(g64 * A0s), k1 = (T)(g64 * (Bd - A0s));
    const T k2 = (T)(g64 * (Cd - Bd)), k3 = (T)(g64 * Cd);
    const T omg = (T)(1.0 - g64);
    const T bx = (T)bx64, by = (T)by64;

    // force term: dF(v) = a + b.v + v.M.v (Sec. III C, App. B)
    T fa = 0, fbx = 0, fby = 0, Mxx = 0, Mxy = 0, Myy = 0, Mzz = 0;
    if constexpr (FORCED) {
        const T E = (T)E64;
        fa = (T)(-0.5) * dt * fma(Fx, m.Jx, Fy * m.Jy);
        fbx = dt * E * Fx;
        fby = dt * E * Fy;
        const T Sxx = fma(Fx, m.Rxxx, Fy * m.Rxxy);
        const T Sxy = fma(Fx, m.Rxxy, Fy * m.Rxyy);
        const T Syy = fma(Fx, m.Rxyy, Fy * m.Ryyy);
        const T k2f = (D == 3 ? (T)2.5 : (T)2.0) * dt;
        Mxx = k2f * fma((T)2 * Fx, m.Jx, -Sxx);
        Mxy = k2f * (fma(Fx, m.Jy, Fy * m.Jx) - Sxy);
        Myy = k2f * fma((T)2 * Fy, m.Jy, -Syy);
        if constexpr (D == 3) {
            const T Rxzz = m.Jx - m.Rxxx - m.Rxyy;   // |v| = 1
            const T Ryzz = m.Jy - m.Rxxy - m.Ryyy;
            Mzz = -k2f * fma(Fx, Rxzz, Fy * Ryzz);
        }
    }

    // (e) collide + force, store:  F' <- (1 - omega) F' + omega (F_eq - shift) + dF
    // For a member with velocity +-v, v = (m d, vz), d one of the in-plane
    // directions X = (1, 0), Y = (0, 1), P = (1, 1), M = (1, -1) (or none), and
    // t = beta.v = m (beta.d):
    //   even part  k0 + fa + k2 t^2 + v.Mf.v = (k0 + fa + vz^2 Mzz) + m^2 SN_d,
    //              SN_d = k2 (beta.d)^2 + d.Mf.d;
    //   odd part   t k1 - k3 t^3 + v.fb     = m (PN_d - k3 m^2 (beta.d)^3),
    //              PN_d = k1 (beta.d) + d.fb;
    //   rate       omega = g (1 - t), so 1 - omega = omg + g m (beta.d).
    // The direction quantities are formed once per site; a class costs a few
    // fused multiply-adds.
    T tn[4] = {bx, by, bx + by, bx - by};
    T SN[4], PN[4], tn3[4];
    T dM[4] = {0, 0, 0, 0}, dfb[4] = {0, 0, 0, 0};
    T k0e = k0, eh = k0, et = k0, ez = k0;   // k0 + fa + vz^2 Mzz for vz^2 = 0, 1/2, 1/3, 1
    if constexpr (FORCED) {
        const T dxy = Mxx + Myy;
        dM[0] = Mxx; dM[1] = Myy;
        dM[2] = fma((T)2, Mxy, dxy); dM[3] = fma((T)-2, Mxy, dxy);
        dfb[0] = fbx; dfb[1] = fby; dfb[2] = fbx + fby; dfb[3] = fbx - fby;
        k0e = k0 + fa;
        eh = fma((T)0.5, Mzz, k0e);
        et = fma((T)(1.0 / 3.0), Mzz, k0e);
        ez = k0e + Mzz;
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const T t2 = tn[d] * tn[d];
        tn3[d] = t2 * tn[d];
        SN[d] = fma(k2, t2, dM[d]);
        PN[d] = fma(k1, tn[d], dfb[d]);
    }
    const T k3m[3] = {k3, k3 * (T)0.5, k3 * (T)(1.0 / 3.0)};                 // k3 m^2
    const T gm[3] = {g, g * (T)kInvSqrt2, g * (T)kInvSqrt3};                // g m
    sfor<0, St::NC>([&](auto ic) {
        constexpr DirClass Cl = St::cls[ic];
        static_assert(Cl.sx >= 0, "class directions are listed with c_x >= 0");
        constexpr int di = Cl.sx != 0 ? (Cl.sy == 0 ? 0 : (Cl.sy > 0 ? 2 : 3)) : (Cl.sy != 0 ? 1 : -1);
        constexpr int mi = Cl.ncomp - 1;
        constexpr double m = comp_mag(Cl.ncomp);
        const T e0 = Cl.vz2 == 0.0 ? k0e : (Cl.vz2 == 0.5 ? eh : (Cl.vz2 == 1.0 ? ez : et));
        if constexpr (di < 0) {
            // v = (0, 0, +-1): t = 0, no odd part, rate omega = g
            sfor<0, Cl.nplus>([&](auto i) {
                constexpr int q = Cl.first + decltype(i)::value;
                fin(std::integral_constant<int, q>{}, omg, f[q], e0);
            });
        } else {
            const T ep = fma((T)(m * m), SN[di], e0);
            const T op = (T)m * fma(-k3m[mi], tn3[di], PN[di]);
            const T Kp = ep + op;
            const T mp = fma(gm[mi], tn[di], omg);
            sfor<0, Cl.nplus>([&](auto i) {
                constexpr int q = Cl.first + decltype(i)::value;
                fin(std::integral_constant<int, q>{}, mp, f[q], Kp);
            });
            if constexpr (Cl.nminus > 0) {
                const T Km = ep - op;
                const T mm = fma(-gm[mi], tn[di], omg);
                sfor<0, Cl.nminus>([&](auto i) {
                    constexpr int q = Cl.first + Cl.nplus + decltype(i)::value;
                    fin(std::integral_constant<int, q>{}, mm, f[q], Km);
                });
            }
        }
    });
}

// sink(qc, r) receives population qc of the new state as the storage value
// r = raw(F_q - shift), the last multiply-add rounded by S::fma_round.
template <class S, class St, bool FORCED, class T, class Sink>
__device__ __forceinline__ void update_site_to(const T (&f)[St::Q], const SiteCtx<T>& ctx, T Fx,
                                               T Fy, Sink&& sink, int* d_flag) {
    update_site_fma<S, St, FORCED>(
        f, ctx, Fx, Fy, [&](auto qc, T a, T b, T c) { sink(qc, S::fma_round(a, b, c)); }, d_flag);
}

// ... storing into global memory: the destination row drow, byte offset own.
// STREAM: non-temporal stores, for lattices far larger than the caches (the
// new state is not read again before the whole lattice has been swept).
template <class S, class St, bool FORCED, bool STREAM = false, class T>
__device__ __forceinline__ void update_site(const T (&f)[St::Q], const SiteCtx<T>& ctx, T Fx,
                                            T Fy, gp<char> drow, uint32_t own, int* d_flag) {
    using raw = typename S::raw;
    constexpr long long plane_bytes = kTileW * sizeof(raw);
    update_site_to<S, St, FORCED>(
        f, ctx, Fx, Fy,
        [&](auto qc, raw r) {
            constexpr int q = decltype(qc)::value;
            const gp<raw> p = (gp<raw>)(drow + (long long)q * plane_bytes + own);
            if constexpr (STREAM) __builtin_nontemporal_store(r, p);
            else *p = r;
        },
        d_flag);
}
}  // namespace rlbm

namespace rlbm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64-bit multiplies by fixed odd constants, high/low halves mixed with
// the other two counter words and the key, key bumped by Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
        const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// ---------------------------------------------------------------------------
// Force table of one time step (paper Sec. V forcing, redrawn every step).
// For row y and k = |kx| in [0, K]:
//   G_kx(y) = sum over the modes with this kx of
//             A r (cos th, sin th) exp(i phi) exp(i 2 pi ky y / ny),
//   P_c(k, y) = Re G_k + Re G_-k,   Q_c(k, y) = Im G_k - Im G_-k,
// so that F_c(x, y) = sum_k cos(2 pi k x/nx) P_c(k, y) - sin(2 pi k x/nx) Q_c(k, y).
// Per mode, Philox4x32-10 with counter (m, step, realization, 0) and key
// seed gives r = u(x0), th = 2 pi u(x1), phi = 2 pi u(x2), u(x) = (x + 1/2) 2^-32.
//
// One work item = one k and the 64*th rows [chunk * 64 th, ...), one row per
// thread of the block.  The draws of up to 64 modes are computed once per
// item by the first wavefront and shared through LDS; exp(i 2 pi ky y / ny)
// comes from the row twiddle table.  Must be called by every thread of the
// block (it synchronises).
// ---------------------------------------------------------------------------
template <class T>
__device__ void force_item(const RealDesc& Dsc, int local_item, int64_t step, int rows) {
    __shared__ T sm_c[64][4];
    __shared__ int sm_ky[64];
    __shared__ T sm_sg[64];
    const int K1 = uni(Dsc.K) + 1;
    const int ny = uni(Dsc.ny);
    const int chunk = local_item / K1;
    const int k = local_item - chunk * K1;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int y = chunk * rows + tid;
    const gp<const T> twy = (gp<const T>)uni((const T*)Dsc.twy);
    const gp<const int> modes = (gp<const int>)uni((const int*)Dsc.modes);   // (kx, ky, m, 0)
    const gp<const int> kptr = (gp<const int>)uni(Dsc.kptr);
    const int j0 = kptr[k], j1 = kptr[k + 1];
    const uint64_t seed = uni(Dsc.seed);
    const uint32_t real = (uint32_t)uni(Dsc.realization);
    const double amp = uni(Dsc.amplitude);
    T Px = 0, Qx = 0, Py = 0, Qy = 0;
    for (int jb = j0; jb < j1; jb += 64) {
        const int nm = min(64, j1 - jb);
        if (tid < nm) {
            const int mkx = modes[4 * (jb + tid)];
            const int mky = modes[4 * (jb + tid) + 1];
            const int mid = modes[4 * (jb + tid) + 2];
            uint32_t c[4] = {(uint32_t)mid, (uint32_t)(uint64_t)step, real, 0u};
            philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            const double u32 = 2.3283064365386963e-10;   // 2^-32
            const double two_pi = 2.0 * M_PI;
            const double rmag = ((double)c[0] + 0.5) * u32;
            const double th = two_pi * (((double)c[1] + 0.5) * u32);
            const double ph = two_pi * (((double)c[2] + 0.5) * u32);
            T ct, st, cph, sph;
            if constexpr (std::is_same<T, double>::value) {
                sincos(th, &st, &ct);
                sincos(ph, &sph, &cph);
            } else {
                sincosf((float)th, &st, &ct);
                sincosf((float)ph, &sph, &cph);
            }
            const T ax = (T)(amp * rmag) * ct, ay = (T)(amp * rmag) * st;
            sm_c[tid][0] = ax * cph;
            sm_c[tid][1] = ax * sph;
            sm_c[tid][2] = ay * cph;
            sm_c[tid][3] = ay * sph;
            sm_ky[tid] = mky;
            sm_sg[tid] = mkx < 0 ? (T)-1 : (T)1;
        }
        __syncthreads();
        if (y < ny) {
            for (int i = 0; i < nm; ++i) {
                const int jy = (int)(((long long)sm_ky[i] * y) % ny);
                T cy, sy;
                if constexpr (std::is_same<T, double>::value) {
                    cy = twy[2 * jy];
                    sy = twy[2 * jy + 1];
                } else {
                    // hardware sine/cosine take the angle in revolutions
                    const float rev = (float)jy / (float)ny;
                    cy = __builtin_amdgcn_cosf(rev);
                    sy = __builtin_amdgcn_sinf(rev);
                }
                // (a + i b) exp(i psi): real a cy - b sy, imaginary b cy + a sy
                Px += fma(sm_c[i][0], cy, -sm_c[i][1] * sy);
                Qx += sm_sg[i] * fma(sm_c[i][1], cy, sm_c[i][0] * sy);
                Py += fma(sm_c[i][2], cy, -sm_c[i][3] * sy);
                Qy += sm_sg[i] * fma(sm_c[i][3], cy, sm_c[i][2] * sy);
            }
        }
        __syncthreads();
    }
    if (y < ny) {
        const gp<T> g = (gp<T>)uni((T*)Dsc.g[(int)(step & 3)]);
        if constexpr (std::is_same<T, double>::value) {
            // [ny][K+1][4] = (Px, Qx, Py, Qy)
            const size_t o = ((size_t)y * K1 + k) * 4;
            g[o + 0] = Px;
            g[o + 1] = Qx;
            g[o + 2] = Py;
            g[o + 3] = Qy;
        } else {
            // [ny][J][2]: term 2k = (Px, Py), term 2k + 1 = (-Qx, -Qy); the terms
            // from 2 (K + 1) to J - 1 stay zero
            const size_t o = (size_t)y * 2 * uni(Dsc.J) + 4 * (size_t)k;
            g[o + 0] = Px;
            g[o + 1] = Py;
            g[o + 2] = -Qx;
            g[o + 3] = -Qy;
        }
    }
}

}  // namespace rlbm
