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
// Only the population loads and stores touch HBM.  After its tiles, every
// block also builds part of the next step's force table.
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
    constexpr bool F64 = std::is_same<T, double>::value;

    const int64_t step = *A.d_step + A.step_off;
    const int par = (int)(step & 1);
    const int lx = threadIdx.x;
    const int ly = threadIdx.y;

    // XCD-aware persistent schedule: XCD x = b mod 8 owns tiles
    // [x * chunk, (x + 1) * chunk); its nb blocks stride through them.
    const int G = A.tile_blocks;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int chunk = (A.n_tiles + 7) >> 3;
    const int t_end = min(A.n_tiles, (xcd + 1) * chunk);

    // per-lattice context, reloaded when the lattice changes (ensembles)
    int cur_r = -1;
    int nx = 0, ny = 0, tiles_x = 1, tile_begin = 0, K = -1;
    int dq = 0, dr = 0;                      // nb = dq * tiles_x + dr
    long long rowq_bytes = 0, plane_bytes = 0;
    const char* src = nullptr;
    char* dst = nullptr;
    InterpW<T> W;
    T ginv = 0, dt = 0;
    const T* twp = nullptr;
    const T* gtab = nullptr;
    int txi = 0, tyi = 0, t_prev = -1;

    for (int t = b < G ? xcd * chunk + (b >> 3) : t_end; t < t_end; t += nb) {
        const int r = A.tile_real ? uni((int)A.tile_real[t]) : 0;
        if (r != cur_r) {
            const RealDesc& Dsc = A.desc[r];
            nx = uni(Dsc.nx);
            ny = uni(Dsc.ny);
            tiles_x = uni(Dsc.tiles_x);
            tile_begin = uni(Dsc.tile_begin);
            const int pitch = uni(Dsc.pitch);
            plane_bytes = (long long)pitch * (long long)sizeof(raw);
            rowq_bytes = plane_bytes * St::Q;
            src = (const char*)uni(Dsc.buf[par]);
            dst = (char*)uni(Dsc.buf[par ^ 1]);
            if constexpr (F64) {
                W.set(uni(Dsc.a[0]), uni(Dsc.a[1]), uni(Dsc.a[2]));
                ginv = uni(Dsc.inv_tau);
                dt = uni(Dsc.dt);
            } else {
                W.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
                ginv = uni(Dsc.inv_tauf);
                dt = uni(Dsc.dtf);
            }
            if constexpr (FORCED) {
                K = uni(Dsc.K);
                twp = uni((const T*)Dsc.twx);
                gtab = uni((const T*)Dsc.g[par]);
            }
            dq = nb / tiles_x;
            dr = nb - dq * tiles_x;
            cur_r = r;
            t_prev = -1;
        }
        // tile coordinates: one division per lattice, then incremental
        if (t_prev < 0) {
            const int local = t - tile_begin;
            tyi = local / tiles_x;
            txi = local - tyi * tiles_x;
        } else {
            txi += dr;
            tyi += dq;
            if (txi >= tiles_x) { txi -= tiles_x; ++tyi; }
        }
        t_prev = t;
        const int x = txi * kTileW + lx;
        const int y = uni(tyi * A.th + ly);          // one tile row per wavefront
        if (x >= nx || y >= ny) continue;

        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1;
        const int yp = y == ny - 1 ? 0 : y + 1;
        const char* const rows[3] = {src + ym * rowq_bytes, src + y * rowq_bytes,
                                     src + yp * rowq_bytes};
        const uint32_t cols[3] = {(uint32_t)(xm * sizeof(raw)), (uint32_t)(x * sizeof(raw)),
                                  (uint32_t)(xp * sizeof(raw))};

        // (b) stream
        T f[St::Q];
        stream_pull<S, St, UNIT>(rows, plane_bytes, cols, W, f);

        // (c) moments, Landau frame in FP64
        const Moments<T> m = moments<St, FORCED>(f);
        const double E64 = (double)m.E + (double)S::shift;
        const double dshift = (double)S::shift / D;     // sum_q w v_i v_i = 1/D per axis
        double eps, bx64, by64;
        const bool ok = landau64<D>(E64, (double)m.Jx, (double)m.Jy,
                                    (double)m.Pxx + dshift, (double)m.Pxy,
                                    (double)m.Pyy + dshift, eps, bx64, by64);
        if (!ok) *A.d_flag = 1;

        // (d) equilibrium F_eq - shift = A0' + B t + C t^2 (t = beta.v), and the
        // Anderson-Witting rate omega = g (1 - t), g = gamma / tau.  For the +v
        // and -v members of a class:
        //   omega (F_eq - shift) = E(t) +- O(t),
        //   E = g A0' + g (C - B) t^2,   O = g (B - A0') t - g C t^3.
        double A0d, Bd, Cd, gam;
        eq_coeffs<D>(eps, bx64, by64, A0d, Bd, Cd, gam);
        const double A0s = A0d - (double)S::shift;
        const double g64 = gam * (double)ginv;
        const T g = (T)g64;
        const T k0 = (T)(g64 * A0s), k1 = (T)(g64 * (Bd - A0s));
        const T k2 = (T)(g64 * (Cd - Bd)), k3 = (T)(g64 * Cd);
        const T omg = (T)(1.0 - g64);
        const T bx = (T)bx64, by = (T)by64;

        // force term: dF(v) = a + b.v + v.M.v (Sec. III C, App. B)
        T fa = 0, fbx = 0, fby = 0, Mxx = 0, Mxy = 0, Myy = 0, Mzz = 0;
        if constexpr (FORCED) {
            // F_c(x, y) = sum_k cos(k a) P_c(k, y) - sin(k a) Q_c(k, y), a = 2 pi x / nx;
            // cos/sin(k a) by the Chebyshev recurrence.
            T Fx = 0, Fy = 0;
            if (K >= 0) {                       // K < 0: this lattice is unforced
                const gp<const T> twx = (gp<const T>)twp;
                const T c1 = twx[2 * x];
                const T s1 = twx[2 * x + 1];
                const gp<const T> grow = (gp<const T>)gtab + (size_t)y * (K + 1) * 4;
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
            const T k2f = (D == 3 ? (T)2.5 : (T)2.0) * dt;
            Mxx = k2f * ((T)2 * Fx * m.Jx - Sxx);
            Mxy = k2f * (Fx * m.Jy + Fy * m.Jx - Sxy);
            Myy = k2f * ((T)2 * Fy * m.Jy - Syy);
            if constexpr (D == 3) {
                const T Rxzz = m.Jx - m.Rxxx - m.Rxyy;   // |v| = 1
                const T Ryzz = m.Jy - m.Rxxy - m.Ryyy;
                Mzz = -k2f * (Fx * Rxzz + Fy * Ryzz);
            }
        }

        // (e) collide + force, store:  F' <- (1 - omega) F' + omega (F_eq - shift) + dF
        const gp<char> drow = (gp<char>)(dst + y * rowq_bytes);
        const uint32_t own = cols[1];
        sfor<0, St::NC>([&](auto ic) {
            constexpr DirClass Cl = St::cls[ic];
            constexpr double um = comp_mag(Cl.ncomp);
            constexpr double ux = Cl.sx * um, uy = Cl.sy * um;
            T t = 0;
            if constexpr (ux != 0.0) t = (T)ux * bx;
            if constexpr (uy != 0.0) t = fma((T)uy, by, t);
            const T t2 = t * t;
            const T Ev = fma(k2, t2, k0);
            const T Ov = t * fma(-k3, t2, k1);
            T dfe = fa, dfo = 0;
            if constexpr (FORCED) {
                if constexpr (ux != 0.0) dfe = fma((T)(ux * ux), Mxx, dfe);
                if constexpr (ux != 0.0 && uy != 0.0) dfe = fma((T)(2.0 * ux * uy), Mxy, dfe);
                if constexpr (uy != 0.0) dfe = fma((T)(uy * uy), Myy, dfe);
                if constexpr (Cl.vz2 != 0.0) dfe = fma((T)Cl.vz2, Mzz, dfe);
                if constexpr (ux != 0.0) dfo = (T)ux * fbx;
                if constexpr (uy != 0.0) dfo = fma((T)uy, fby, dfo);
            }
            const T ep = Ev + dfe;
            const T op = Ov + dfo;
            const T gt = g * t;
            const T Kp = ep + op;
            const T mp = omg + gt;
            sfor<0, Cl.nplus>([&](auto i) {
                constexpr int q = Cl.first + decltype(i)::value;
                S::st((gp<raw>)(drow + (long long)q * plane_bytes + own), fma(mp, f[q], Kp));
            });
            if constexpr (Cl.nminus > 0) {
                const T Km = ep - op;
                const T mm = omg - gt;
                sfor<0, Cl.nminus>([&](auto i) {
                    constexpr int q = Cl.first + Cl.nplus + decltype(i)::value;
                    S::st((gp<raw>)(drow + (long long)q * plane_bytes + own), fma(mm, f[q], Km));
                });
            }
        });
    }

    // force table of the next step: on the extra blocks when there are any,
    // else the items of each XCD spread over its tile blocks
    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        const int u0 = extra > 0 ? b - G : xcd + 8 * (b >> 3);
        const int du = extra > 0 ? extra : 8 * nb;
        for (int u = u0 >= 0 ? u0 : A.n_gitems; u < A.n_gitems; u += du) {
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
