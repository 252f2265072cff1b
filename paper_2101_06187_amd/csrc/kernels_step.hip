// The fused RLBM time step (paper Sec. III C, algorithm (b)-(e), with the
// stirring force of Sec. III C / App. B), one translation unit per storage
// form, selected by RLBM_STORAGE_ID at compile time.
//
// One thread owns one lattice site.  A block is a tile of 64 x th sites (one
// wavefront per tile row).  The grid is persistent: block b walks the tiles of
// the chunk that belongs to its XCD (b mod 8), so horizontally and vertically
// adjacent tiles -- which share halo cache lines -- are served by the same L2.
// Per site, in registers:
//   stream (pull, bilinear)  ->  moments  ->  FP64 Landau frame  ->
//   equilibrium coefficients ->  force field + projected force term  ->
//   Anderson-Witting collision  ->  store.
// Only the population loads and stores touch HBM.
#include <hip/hip_ext.h>

#include "site.hpp"

#ifndef RLBM_STORAGE_ID
#error "RLBM_STORAGE_ID must be defined"
#endif

namespace rlbm {

#if RLBM_STORAGE_ID == 0
using Store = StF64;
#elif RLBM_STORAGE_ID == 1
using Store = StF32;
#elif RLBM_STORAGE_ID == 2
using Store = StF16S;
#else
using Store = StBF16S;
#endif

template <class S, class St, bool UNIT, bool FORCED>
__global__ __launch_bounds__(512) void step_kernel(StepArgs A) {
    using T = typename S::T;
    using raw = typename S::raw;
    constexpr int D = St::D;
    constexpr T sig = (T)S::shift;

    const int64_t step = *A.d_step + A.step_off;
    const int par = (int)(step & 1);
    const int lx = threadIdx.x;
    const int ly = threadIdx.y;

    // XCD-aware persistent schedule
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int chunk = (A.n_tiles + 7) >> 3;
    const int t_end = min(A.n_tiles, (xcd + 1) * chunk);

    for (int t = xcd * chunk + (b >> 3); t < t_end; t += nb) {
        const int r = A.tile_real ? uni((int)A.tile_real[t]) : 0;
        const RealDesc& Dsc = A.desc[r];
        const int nx = uni(Dsc.nx), ny = uni(Dsc.ny);
        const int tiles_x = uni(Dsc.tiles_x);
        const int local = t - uni(Dsc.tile_begin);
        const int tyi = local / tiles_x;
        const int txi = local - tyi * tiles_x;
        const int x = txi * kTileW + lx;
        const int y = tyi * A.th + ly;
        if (x >= nx || y >= ny) continue;

        const int pitch = uni(Dsc.pitch);
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1;
        const int yp = y == ny - 1 ? 0 : y + 1;
        const int rows[3] = {ym * pitch, y * pitch, yp * pitch};
        const int cols[3] = {xm, x, xp};
        uint32_t off[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) off[j][i] = (uint32_t)(rows[j] + cols[i]) * sizeof(raw);

        const long long plane_bytes = uni(Dsc.plane) * (long long)sizeof(raw);
        const char* src = (const char*)uni(Dsc.buf[par]);
        char* dst = (char*)uni(Dsc.buf[par ^ 1]);

        T a1, a2, a3;
        if constexpr (std::is_same<T, double>::value) {
            a1 = uni(Dsc.a[0]); a2 = uni(Dsc.a[1]); a3 = uni(Dsc.a[2]);
        } else {
            a1 = uni(Dsc.af[0]); a2 = uni(Dsc.af[1]); a3 = uni(Dsc.af[2]);
        }

        // (b) stream
        T f[St::Q];
        stream_pull<S, St, UNIT>(src, plane_bytes, off, a1, a2, a3, f);

        // (c) moments, Landau frame in FP64
        const Moments<T> m = moments<St, FORCED>(f);
        const double E64 = (double)m.E + (double)S::shift;
        const double dshift = (double)S::shift / D;     // sum_q w v_i v_i = 1/D per axis
        double eps, bx64, by64;
        const bool ok = landau64<D>(E64, (double)m.Jx, (double)m.Jy,
                                    (double)m.Pxx + dshift, (double)m.Pxy,
                                    (double)m.Pyy + dshift, eps, bx64, by64);
        if (!ok) *A.d_flag = 1;

        // (d) equilibrium coefficients
        double A0d, Bd, Cd, gam;
        eq_coeffs<D>(eps, bx64, by64, A0d, Bd, Cd, gam);
        const T A0 = (T)(A0d - (double)S::shift);
        const T B = (T)Bd, C = (T)Cd;
        const T g = std::is_same<T, double>::value ? (T)(gam * uni(Dsc.inv_tau))
                                                   : (T)gam * uni(Dsc.inv_tauf);
        const T bx = (T)bx64, by = (T)by64;

        // force term coefficients: dF(v) = a + b.v + v.M.v (Sec. III C, App. B)
        T fa = 0, fbx = 0, fby = 0, Mxx = 0, Mxy = 0, Myy = 0, Mzz = 0;
        if constexpr (FORCED) {
            const T dt = std::is_same<T, double>::value ? (T)uni(Dsc.dt) : (T)uni(Dsc.dtf);
            // configuration-space force: F_c(x, y) = sum_k cos(k a) P_c(k, y) - sin(k a) Q_c(k, y)
            // with a = 2 pi x / nx; cos/sin(k a) by the Chebyshev recurrence.
            T Fx = 0, Fy = 0;
            const int K = uni(Dsc.K);          // -1: this lattice is unforced (no table)
            if (K >= 0) {
                const int yu = uni(y);         // one tile row per wavefront
                const gp<const T> twx = (gp<const T>)uni((const T*)Dsc.twx);
                const T c1 = twx[2 * x];
                const T s1 = twx[2 * x + 1];
                const gp<const T> grow =
                    (gp<const T>)uni((const T*)Dsc.g[par]) + (size_t)yu * (K + 1) * 4;
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
                int k = 1;
                for (; k + 3 <= K; k += 4) {      // four table rows per batch of loads
                    T gv[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) gv[i] = grow[4 * k + i];
#pragma unroll
                    for (int i = 0; i < 4; ++i) term(gv[4 * i], gv[4 * i + 1], gv[4 * i + 2], gv[4 * i + 3]);
                }
                for (; k <= K; ++k) term(grow[4 * k], grow[4 * k + 1], grow[4 * k + 2], grow[4 * k + 3]);
            }
            const T E = (T)E64;
            fa = (T)(-0.5) * dt * (Fx * m.Jx + Fy * m.Jy);
            fbx = dt * E * Fx;
            fby = dt * E * Fy;
            const T Sxx = Fx * m.Rxxx + Fy * m.Rxxy;
            const T Sxy = Fx * m.Rxxy + Fy * m.Rxyy;
            const T Syy = Fx * m.Rxyy + Fy * m.Ryyy;
            const T k2 = (D == 3 ? (T)2.5 : (T)2.0) * dt;
            Mxx = k2 * ((T)2 * Fx * m.Jx - Sxx);
            Mxy = k2 * (Fx * m.Jy + Fy * m.Jx - Sxy);
            Myy = k2 * ((T)2 * Fy * m.Jy - Syy);
            if constexpr (D == 3) {
                const T Rxzz = m.Jx - m.Rxxx - m.Rxyy;   // |v| = 1
                const T Ryzz = m.Jy - m.Rxxy - m.Ryyy;
                Mzz = -k2 * (Fx * Rxzz + Fy * Ryzz);
            }
        }

        // (e) collide + force, store
        const uint32_t own = off[1][1];
        const gp<char> gdst = (gp<char>)dst;
        sfor<0, St::NC>([&](auto ic) {
            constexpr DirClass Cl = St::cls[ic];
            constexpr double um = comp_mag(Cl.ncomp);
            constexpr double ux = Cl.sx * um, uy = Cl.sy * um;
            T t = 0;
            if constexpr (ux != 0.0) t = (T)ux * bx;
            if constexpr (uy != 0.0) t = fma((T)uy, by, t);
            const T feq_e = fma(C, t * t, A0);
            const T feq_o = B * t;
            const T gt = g * t;
            const T wp = g - gt, wm = g + gt;
            T dfe = fa, dfo = 0;
            if constexpr (FORCED) {
                if constexpr (ux != 0.0) dfe = fma((T)(ux * ux), Mxx, dfe);
                if constexpr (ux != 0.0 && uy != 0.0) dfe = fma((T)(2.0 * ux * uy), Mxy, dfe);
                if constexpr (uy != 0.0) dfe = fma((T)(uy * uy), Myy, dfe);
                if constexpr (Cl.vz2 != 0.0) dfe = fma((T)Cl.vz2, Mzz, dfe);
                if constexpr (ux != 0.0) dfo = (T)ux * fbx;
                if constexpr (uy != 0.0) dfo = fma((T)uy, fby, dfo);
            }
            const T Kp = fma(wp, feq_e + feq_o, dfe + dfo);
            const T mp = (T)1 - wp;
            sfor<0, Cl.nplus>([&](auto i) {
                constexpr int q = Cl.first + decltype(i)::value;
                S::st((gp<raw>)(gdst + (long long)q * plane_bytes + own), fma(mp, f[q], Kp));
            });
            if constexpr (Cl.nminus > 0) {
                const T Km = fma(wm, feq_e - feq_o, dfe - dfo);
                const T mm = (T)1 - wm;
                sfor<0, Cl.nminus>([&](auto i) {
                    constexpr int q = Cl.first + Cl.nplus + decltype(i)::value;
                    S::st((gp<raw>)(gdst + (long long)q * plane_bytes + own), fma(mm, f[q], Km));
                });
            }
        });
        (void)sig;
    }

    // force table of the next step: items of this XCD, spread over its blocks
    if constexpr (FORCED) {
        for (int u = xcd + 8 * (b >> 3); u < A.n_gitems; u += 8 * nb) {
            const int r = A.gitem_real ? uni((int)A.gitem_real[u]) : 0;
            const RealDesc& Dsc = A.desc[r];
            force_item<T>(Dsc, u - uni(Dsc.gitem_begin), step + 1, kTileW * A.th);
        }
    }
}

template <class St, bool UNIT, bool FORCED>
static const void* kernel_ptr() {
    return (const void*)step_kernel<Store, St, UNIT, FORCED>;
}

static const void* select_kernel(int stencil, bool unit, bool forced) {
    if (stencil == RLBM_STENCIL_SPH26) {
        if (unit) return forced ? kernel_ptr<Sph26, true, true>() : kernel_ptr<Sph26, true, false>();
        return forced ? kernel_ptr<Sph26, false, true>() : kernel_ptr<Sph26, false, false>();
    }
    if (unit) return forced ? kernel_ptr<Circ8, true, true>() : kernel_ptr<Circ8, true, false>();
    return forced ? kernel_ptr<Circ8, false, true>() : kernel_ptr<Circ8, false, false>();
}

#if RLBM_STORAGE_ID == 0
#define RLBM_LAUNCH_NAME launch_step_f64
#define RLBM_OCC_NAME occ_f64
#elif RLBM_STORAGE_ID == 1
#define RLBM_LAUNCH_NAME launch_step_f32
#define RLBM_OCC_NAME occ_f32
#elif RLBM_STORAGE_ID == 2
#define RLBM_LAUNCH_NAME launch_step_f16s
#define RLBM_OCC_NAME occ_f16s
#else
#define RLBM_LAUNCH_NAME launch_step_bf16s
#define RLBM_OCC_NAME occ_bf16s
#endif

hipError_t RLBM_LAUNCH_NAME(const StepLaunch& L) {
    const void* k = select_kernel(L.stencil, L.unit_cfl, L.forced);
    StepArgs a = L.args;
    void* params[] = {&a};
    if (L.ev_start)
        return hipExtLaunchKernel(k, dim3(L.grid), dim3(kTileW, L.args.th), params, 0, L.stream,
                                  L.ev_start, L.ev_stop, 0);
    return hipLaunchKernel(k, dim3(L.grid), dim3(kTileW, L.args.th), params, 0, L.stream);
}

int RLBM_OCC_NAME(int stencil, bool unit, bool forced, int th) {
    int blocks = 0;
    const void* k = select_kernel(stencil, unit, forced);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, kTileW * th, 0) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace rlbm
