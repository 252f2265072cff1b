// The fused RLBM time step (paper Sec. III C, algorithm (b)-(e), with the
// stirring force of Sec. III C / App. B), one translation unit per storage
// form, selected by RLBM_STORAGE_ID at compile time.
//
// Five forms of the same per-site update (update_site in site.hpp):
//   step_kernel       -- one thread owns one lattice site; a block is a tile
//                        of 64 x th sites (one wavefront per tile row);
//   staged_kernel     -- the same tile with every population row it needs
//                        staged in LDS once;
//   march_kernel      -- a wavefront marches down a 64-column strip segment
//                        with a rolling register window of rows;
//   march_pair_kernel -- the same with two columns per lane (16-bit storage);
//   march2_kernel     -- the marching form for two time steps per launch.
// Grids are persistent: block b walks the work items of the chunk that belongs
// to its XCD (b mod 8), so adjacent tiles -- which share halo cache lines --
// are served by the same L2.  Per site, in registers:
//   stream (pull, bilinear)  ->  moments  ->  FP64 Landau frame  ->
//   equilibrium coefficients ->  force field + projected force term  ->
//   Anderson-Witting collision  ->  store.
// Only the population loads and stores touch HBM.  Blocks without tiles (or,
// when there are none, every block after its tiles) build the force tables of
// the two steps after the launch.
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

// Force tables of the steps after this launch (s + nsteps and the one after
// it): 2 n_gitems items; this block takes items u0, u0 + du, ...
template <class T>
__device__ __forceinline__ void build_force_tables(const StepArgs& A, int64_t step, int u0, int du) {
    const int n = A.n_gitems;
    for (int v = u0 >= 0 ? u0 : 2 * n; v < 2 * n; v += du) {
        const int second = v >= n;
        const int u = second ? v - n : v;
        const int r = A.gitem_real ? uni((int)A.gitem_real[u]) : 0;
        const RealDesc& Dsc = A.desc[r];
        force_item<T>(Dsc, u - uni(Dsc.wm[A.map].gitem_begin), step + A.nsteps + second,
                      kTileW * A.th);
    }
}

// ---------------------------------------------------------------------------
// Stirring force of the FP32 forms (force_chunk in site.hpp): the marching
// forms keep the force basis of their strip in LDS, [J/4][W][4] floats (the
// float4 at g W + col holds terms 4 g .. 4 g + 3 of strip column col), shared
// by the four wavefronts of a block, which march down consecutive segments of
// one strip.  Coefficient registers: kCoefRegs chunks of 16 terms (2 K + 2 <=
// 16 kCoefRegs, i.e. K <= 63) are loaded one row iteration ahead of their
// use; longer sums load the rest where they are used.
// ---------------------------------------------------------------------------
extern __shared__ v4f lds_basis[];
constexpr int kCoefRegs = 8;

// The basis of columns colx(0 .. W-1), block-cooperative.
template <class ColX>
__device__ __forceinline__ void stage_basis(const float* bas, int J, int W, ColX&& colx) {
    const int tid = (int)(threadIdx.y * blockDim.x + threadIdx.x);
    const int nt = (int)(blockDim.x * blockDim.y);
    const int G = J >> 2;
    const gp<const v4f> b4 = (gp<const v4f>)bas;
    for (int f = tid; f < G * W; f += nt) {
        const int g = f / W, col = f - g * W;
        lds_basis[f] = b4[(size_t)colx(col) * G + g];
    }
}

// Coefficient registers of the rows rowA (outputs 0, 1) and rowB (2, 3).
__device__ __forceinline__ void load_coefs(float (&cf)[kCoefRegs], const float* rowA,
                                           const float* rowB, int nch, const ForceLane& fl) {
    const gp<const float> row = (gp<const float>)(fl.hi ? rowB : rowA) + fl.off;
#pragma unroll
    for (int c = 0; c < kCoefRegs; ++c)
        if (c < nch) cf[c] = row[kForceChunk * 2 * c];
}

// The four sums over jt terms of this lane's strip column col (basis in LDS,
// W columns); nch = ceil(jt / 16) chunks.
__device__ __forceinline__ v4f force_sum_lds(const float (&cf)[kCoefRegs], const float* rowA,
                                             const float* rowB, int jt, int col, int W,
                                             const ForceLane& fl) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int nch = (jt + kForceChunk - 1) / kForceChunk;
    const int tail = force_tail(jt);
    auto basis = [&](int c, v4f (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = lds_basis[(4 * c + i) * W + col];
    };
#pragma unroll
    for (int c = 0; c < kCoefRegs; ++c) {
        if (c + 1 < nch) {
            v4f b[4];
            basis(c, b);
            acc = force_chunk(acc, cf[c], b);
        } else if (c + 1 == nch) {
            v4f b[4];
            basis(c, b);
            acc = force_chunk_n(acc, cf[c], b, tail);
        }
    }
    if (nch > kCoefRegs) {
        const gp<const float> row = (gp<const float>)(fl.hi ? rowB : rowA) + fl.off;
        for (int c = kCoefRegs; c < nch; ++c) {
            v4f b[4];
            basis(c, b);
            acc = force_chunk_n(acc, row[kForceChunk * 2 * c], b, c + 1 < nch ? kForceChunk : tail);
        }
    }
    return acc;
}

// The same sums by FP32 fused multiply-adds on the vector ALU, in the same
// term order (each MFMA above is one fused multiply-add per output, so the
// results are bitwise those of the matrix-core sums): the coefficients of one
// table row as constant memory (scalar loads, SGPRs), the basis of the nc
// strip columns cols[0 .. nc-1] from LDS; F[2 i], F[2 i + 1] = (Fx, Fy) of
// column cols[i].  For the one-step marching forms, whose wavefronts issue far
// more vector-ALU work per force sum than the two-step form.
template <int NC>
__device__ __forceinline__ void force_sum_valu(const float* row, int jt, const int (&cols)[NC],
                                               int W, float (&F)[2 * NC]) {
    const kp<const float> r = (kp<const float>)row;
#pragma unroll
    for (int i = 0; i < 2 * NC; ++i) F[i] = 0.f;
    const int nch = (jt + kForceChunk - 1) / kForceChunk;
    // chunk c, its first n terms
    auto chunk = [&](int c, auto all, int n) {
        float cv[2 * kForceChunk];
#pragma unroll
        for (int i = 0; i < 2 * kForceChunk; ++i) cv[i] = r[2 * kForceChunk * c + i];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            v4f b[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) b[k] = lds_basis[(4 * c + g) * W + cols[k]];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * g + i;
                if (decltype(all)::value || t < n) {
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        F[2 * k] = fmaf(cv[2 * t], b[k][i], F[2 * k]);
                        F[2 * k + 1] = fmaf(cv[2 * t + 1], b[k][i], F[2 * k + 1]);
                    }
                }
            }
        }
    };
    for (int c = 0; c + 1 < nch; ++c) chunk(c, std::true_type{}, kForceChunk);
    chunk(nch - 1, std::false_type{}, force_tail(jt));
}

// Work items of the marching forms: a block's four wavefronts take four
// consecutive segments of one strip (they share the strip's force basis);
// consecutive blocks take the next strip of the same rows, so the wavefronts
// running at a time spread over the columns of a band of rows (as the rows of
// one strip, 64 columns apart in the brick layout, would all map to the same
// memory channels).  The segment count of a strip is padded to a multiple of
// 4; a padding item has no rows.
struct MarchItem {
    int strip, seg, ya, yb;
    bool rows;
    __device__ void decode(int local, int strips, int ny, int seglen) {
        const int segs = (ny + seglen - 1) / seglen;
        const int grp = local >> 2;
        const int band = grp / strips;
        strip = grp - band * strips;
        seg = 4 * band + (local & 3);
        rows = seg < segs;
        ya = seg * seglen;
        yb = min(ny, ya + seglen);
    }
    // The two-step form: a block's eight wavefronts take g adjacent strips x
    // 8 / g consecutive segments (strip g p + w % g, segment (8 / g) b + w / g;
    // g = 1, 2 or 4 per lattice), so that the wavefronts marching side by side
    // on one compute unit share the cache lines at their strips' common
    // edges; the strip count is padded to a multiple of g, the segment count
    // of a strip to a multiple of 8 / g (padding items have no rows).
    __device__ void decode_group(int local, int strips, int g, int ny, int seglen) {
        const int segs = (ny + seglen - 1) / seglen;
        const int sgroups = (strips + g - 1) / g;
        const int grp = local >> 3;
        const int band = grp / sgroups;
        const int w = local & 7;
        const int gw = w / g;                     // g is 1, 2 or 4
        strip = g * (grp - band * sgroups) + (w - gw * g);
        seg = (8 / g) * band + gw;
        rows = seg < segs && strip < strips;
        ya = seg * seglen;
        yb = min(ny, ya + seglen);
    }
};

// The tile form.  With 16-bit storage at cfl = 1 it is held to five
// wavefronts per SIMD (96 VGPRs): its blocks are 64 x th lanes, so residency
// moves in single wavefronts.
template <class S, int SM>
constexpr int tile_min_waves() { return sizeof(typename S::raw) == 2 && SM == kStreamUnit ? 5 : 1; }

template <class S, class St, int SM, bool FORCED>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(tile_min_waves<S, SM>())))
void step_kernel(StepArgs A) {
    using T = typename S::T;
    using raw = typename S::raw;
    constexpr int D = St::D;
    constexpr bool F64 = std::is_same<T, double>::value;

    constexpr bool MF = FORCED && !F64;       // FP32 force sums on the matrix cores

    const int64_t step = A.d_step[0] + A.step_off;
    const int par = (int)((A.d_step[1] + A.launch_off) & 1);
    const int lx = threadIdx.x;
    const int ly = threadIdx.y;
    ForceLane fl;
    fl.init(lx);

    // XCD-aware persistent schedule: XCD x = b mod 8 owns tiles
    // [x * chunk, (x + 1) * chunk); its nb blocks stride through them.
    const int G = A.tile_blocks;
    // The force-table blocks take the first block indices in the FP32 and
    // 16-bit forms: a table item is a longer chain than a tile, and started
    // first it ends within the tiles' single round (b < 0: a table block)
    constexpr bool kTablesFirst = !F64;
    const int b = kTablesFirst ? (int)blockIdx.x - ((int)gridDim.x - G) : (int)blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int chunk = (A.n_tiles + 7) >> 3;
    const int t_end = min(A.n_tiles, (xcd + 1) * chunk);

    // per-lattice context, reloaded when the lattice changes (ensembles)
    int cur_r = -1;
    int nx = 0, ny = 0, tiles_x = 1, tile_begin = 0, K = -1, J = 0;
    const float* bas = nullptr;
    int dq = 0, dr = 0;                      // nb = dq * tiles_x + dr
    long long rowq_bytes = 0;
    const char* src = nullptr;
    char* dst = nullptr;
    InterpW<T> W;
    InterpW2<T> W2;
    T ginv = 0, dt = 0;
    int eta_s = 0;
    const T* twp = nullptr;
    const T* gtab = nullptr;
    int txi = 0, tyi = 0, t_prev = -1;

    for (int t = (kTablesFirst ? b >= 0 : b < G) ? xcd * chunk + (b >> 3) : t_end; t < t_end; t += nb) {
        const int r = A.tile_real ? uni((int)A.tile_real[t]) : 0;
        if (r != cur_r) {
            const RealDesc& Dsc = A.desc[r];
            nx = uni(Dsc.nx);
            ny = uni(Dsc.ny);
            tiles_x = uni(Dsc.wm[A.map].tiles_x);
            tile_begin = uni(Dsc.wm[A.map].tile_begin);
            const int pitch = uni(Dsc.pitch);
            rowq_bytes = (long long)pitch * St::Q * (long long)sizeof(raw);
            src = (const char*)uni(Dsc.buf[par]);
            dst = (char*)uni(Dsc.buf[par ^ 1]);
            if constexpr (F64) {
                if constexpr (SM == kStreamHalo2) W2.set(uni(Dsc.a[0]), uni(Dsc.a[1]), uni(Dsc.a[2]));
                else W.set(uni(Dsc.a[0]), uni(Dsc.a[1]), uni(Dsc.a[2]));
                ginv = uni(Dsc.inv_tau);
                dt = uni(Dsc.dt);
            } else {
                if constexpr (SM == kStreamHalo2) W2.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
                else W.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
                ginv = uni(Dsc.inv_tauf);
                dt = uni(Dsc.dtf);
            }
            eta_s = uni(Dsc.tau_mode);
            if constexpr (FORCED) {
                K = uni(Dsc.K);
                twp = uni((const T*)Dsc.twx);
                gtab = uni((const T*)Dsc.g[step & 3]);
                if constexpr (MF) {
                    J = uni(Dsc.J);
                    bas = uni(Dsc.bas);
                }
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
        if (y >= ny) continue;
        // FP32 force sum with every lane of the wavefront (lanes past the
        // lattice take its last column)
        T Fx = 0, Fy = 0;
        if constexpr (MF) {
            if (K >= 0) {
                const float* row = (const float*)gtab + (size_t)y * 2 * J;
                const v4f acc = force_sum_global(row, row, bas + (size_t)min(x, nx - 1) * J,
                                                 2 * (K + 1), fl);
                Fx = acc[0];
                Fy = acc[1];
            }
        }
        if (x >= nx) continue;

        // (b) stream
        T f[St::Q];
        if constexpr (SM == kStreamHalo2) {
            // rows y-2 .. y+2 and columns x-2 .. x+2, periodic (nx, ny >= 2)
            auto wrap = [](int v, int n) { return v < 0 ? (v + n < 0 ? v + 2 * n : v + n)
                                                        : (v >= n ? (v - n >= n ? v - 2 * n : v - n) : v); };
            const char* rows5[5];
            uint32_t cols5[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                rows5[j] = src + (long long)uni(wrap(y + j - 2, ny)) * rowq_bytes;
                cols5[j] = col_bytes<raw>(wrap(x + j - 2, nx), St::Q);
            }
            stream_pull_h2<S, St>(rows5, cols5, W2, f);
        } else {
            const int xm = x == 0 ? nx - 1 : x - 1;
            const int xp = x == nx - 1 ? 0 : x + 1;
            const int ym = y == 0 ? ny - 1 : y - 1;
            const int yp = y == ny - 1 ? 0 : y + 1;
            const char* const rows[3] = {src + ym * rowq_bytes, src + y * rowq_bytes,
                                         src + yp * rowq_bytes};
            const uint32_t cols[3] = {col_bytes<raw>(xm, St::Q), col_bytes<raw>(x, St::Q),
                                      col_bytes<raw>(xp, St::Q)};
            stream_pull<S, St, SM>(rows, cols, W, f);
        }

        const SiteCtx<T> sctx{ginv, dt, K, gtab, eta_s};
        if constexpr (FORCED && F64) {
            if (K >= 0) {
                const gp<const T> twx = (gp<const T>)twp;
                force_cheb64(sctx, twx[2 * x], twx[2 * x + 1], y, Fx, Fy);
            }
        }
        update_site<S, St, FORCED>(f, sctx, Fx, Fy, (gp<char>)(dst + y * rowq_bytes), col_bytes<raw>(x, St::Q),
                                   A.d_flag);
    }

    // force table of the next step: on the extra blocks when there are any,
    // else the items of each XCD spread over its tile blocks
    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        const int u0 = kTablesFirst ? (b < 0 ? b + extra : -1) : b - G;
        build_force_tables<T>(A, step, extra > 0 ? u0 : xcd + 8 * (b >> 3),
                              extra > 0 ? extra : 8 * nb);
    }
}

// ---------------------------------------------------------------------------
// LDS-staged tile form.  A block of kStageTH wavefronts owns a tile of 64 x
// kStageTH sites.  Every population row the tile needs is read from global
// memory once, with aligned row loads, into LDS: the tile's own rows (every
// population), the row above it (only the populations pulled from above,
// c_y > 0) and the row below it (c_y < 0), each with the two halo columns of
// the strip (one gathered load per row).  After a barrier every site
// interpolates from LDS and applies the same update_site as the other forms,
// so all forms give bitwise identical results.
// In LDS a row is population-major, with the populations ordered by c_y
// (c_y < 0, then c_y = 0, then c_y > 0), so the two partial halo rows take
// only the slots they use: population q of LDS row r (lattice row y0 - 1 + r)
// sits in slot row  r Q + slot(q) - (nD + n0), and a slot row holds kLdsW
// values: halo column x0 - 1 at index 3, the strip's columns at 4 .. 67, the
// right halo column right after the strip's last column.
// ---------------------------------------------------------------------------
constexpr int kStageTH = 4;
constexpr int kLdsW = 72;

template <class St>
struct StageMap {
    static constexpr int Q = St::Q;
    static constexpr int cx(int q) { return St::dir[q].cx; }
    static constexpr int cy(int q) { return St::dir[q].cy; }
    static constexpr int ygroup(int q) { return cy(q) < 0 ? 0 : (cy(q) == 0 ? 1 : 2); }
    static constexpr int count(int g) {
        int n = 0;
        for (int q = 0; q < Q; ++q) n += ygroup(q) == g;
        return n;
    }
    static constexpr int nD = count(0), n0 = count(1), nU = count(2);
    static constexpr int slot(int q) {
        int k = 0;
        for (int p = 0; p < Q; ++p)
            k += ygroup(p) < ygroup(q) || (ygroup(p) == ygroup(q) && p < q);
        return k;
    }
    static constexpr int kSlotRows = kStageTH * Q + nU + nD;
    static constexpr int srow(int r, int q) { return r * Q + slot(q) - (nD + n0); }
    // lanes of the halo gather: populations with c_x != 0
    static constexpr int nH() {
        int k = 0;
        for (int q = 0; q < Q; ++q) k += cx(q) != 0;
        return k;
    }
    static constexpr int hidx(int q) {
        int k = 0;
        for (int p = 0; p < q; ++p) k += cx(p) != 0;
        return k;
    }
};

// FP64 stages twice the bytes (two blocks per CU fit the LDS) and needs its
// registers; the other forms are held to 128 VGPRs, so that four blocks -- one
// tile row per SIMD each -- are resident per CU.
template <class S>
constexpr int stage_min_waves() { return sizeof(typename S::raw) == 8 ? 1 : 4; }

template <class S, class St, int SM, bool FORCED>
__global__ __launch_bounds__(64 * kStageTH, stage_min_waves<S>()) void staged_kernel(StepArgs A) {
    static_assert(SM != kStreamHalo2, "the staged form streams from the nearest rows only");
    using T = typename S::T;
    using raw = typename S::raw;
    using M = StageMap<St>;
    constexpr int Q = St::Q;
    constexpr int TH = kStageTH;
    constexpr bool F64 = std::is_same<T, double>::value;
    constexpr long long plane_bytes = kTileW * sizeof(raw);
    __shared__ raw sm[M::kSlotRows * kLdsW];

    const int64_t step = A.d_step[0] + A.step_off;
    const int par = (int)((A.d_step[1] + A.launch_off) & 1);
    constexpr bool MF = FORCED && !F64;       // FP32 force sums on the matrix cores
    const int lx = threadIdx.x;
    const int w = uni((int)threadIdx.y);
    ForceLane fl;
    fl.init(lx);

    // XCD-aware persistent schedule, as in step_kernel
    const int G = A.tile_blocks;
    // The force-table blocks take the first block indices in the FP32 and
    // 16-bit forms: a table item is a longer chain than a tile, and started
    // first it ends within the tiles' single round (b < 0: a table block)
    constexpr bool kTablesFirst = !F64;
    const int b = kTablesFirst ? (int)blockIdx.x - ((int)gridDim.x - G) : (int)blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int chunk = (A.n_tiles + 7) >> 3;
    const int t_end = min(A.n_tiles, (xcd + 1) * chunk);

    // this lane's population in the halo gather
    int my_q = 0, my_slot = 0, my_cy = 0;
    bool my_left = true;
    sfor<0, Q>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        if constexpr (M::cx(q) != 0) {
            if (lx == M::hidx(q)) {
                my_q = q;
                my_slot = M::slot(q);
                my_cy = M::cy(q);
                my_left = M::cx(q) > 0;
            }
        }
    });

    int cur_r = -1;
    int nx = 0, ny = 0, tiles_x = 1, tile_begin = 0, K = -1, J = 0;
    const float* bas = nullptr;
    long long rowq_bytes = 0;
    const char* src = nullptr;
    char* dst = nullptr;
    InterpW<T> W;
    T ginv = 0, dt = 0;
    int eta_s = 0;
    const T* twp = nullptr;
    const T* gtab = nullptr;

    for (int t = (kTablesFirst ? b >= 0 : b < G) ? xcd * chunk + (b >> 3) : t_end; t < t_end; t += nb) {
        const int r = A.tile_real ? uni((int)A.tile_real[t]) : 0;
        if (r != cur_r) {
            const RealDesc& Dsc = A.desc[r];
            nx = uni(Dsc.nx);
            ny = uni(Dsc.ny);
            tiles_x = uni(Dsc.wm[A.map].tiles_x);
            tile_begin = uni(Dsc.wm[A.map].tile_begin);
            rowq_bytes = (long long)uni(Dsc.pitch) * Q * (long long)sizeof(raw);
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
            eta_s = uni(Dsc.tau_mode);
            if constexpr (FORCED) {
                K = uni(Dsc.K);
                twp = uni((const T*)Dsc.twx);
                gtab = uni((const T*)Dsc.g[step & 3]);
                if constexpr (MF) {
                    J = uni(Dsc.J);
                    bas = uni(Dsc.bas);
                }
            }
            cur_r = r;
        }
        const int local = t - tile_begin;
        const int tyi = local / tiles_x;
        const int x0 = (local - tyi * tiles_x) * kTileW;
        const int y0 = tyi * TH;
        const int R = min(kTileW - 1, nx - 1 - x0);          // last column lane
        const int hcol = my_left ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + R + 1 == nx ? 0 : x0 + R + 1);
        const int hidx = my_left ? 3 : 5 + R;                // LDS index of the halo column
        const uint32_t colb = col_bytes<raw>(x0 + lx, Q);
        const uint32_t hcolb = col_bytes<raw>(hcol, Q);
        auto wrapy = [&](int v) {
            if (v < 0) v += ny;
            if (v >= ny) v -= ny;
            return v >= ny ? v % ny : v;
        };

        // (b) stage LDS row rr = lattice row y0 - 1 + rr: the populations of
        // group g (0: c_y < 0, 1: all, 2: c_y > 0) and their halo columns
        auto stage = [&](int rr, auto gc) {
            constexpr int g = decltype(gc)::value;
            const char* rowp = src + (long long)wrapy(y0 - 1 + rr) * rowq_bytes;
            if (lx <= R) {
                sfor<0, Q>([&](auto iq) {
                    constexpr int q = decltype(iq)::value;
                    if constexpr (g == 1 || M::ygroup(q) == g)
                        sm[M::srow(rr, q) * kLdsW + 4 + lx] =
                            *(gp<const raw>)(rowp + (long long)q * plane_bytes + colb);
                });
            }
            const bool mine = lx < M::nH() && (g == 1 || (g == 0 ? my_cy < 0 : my_cy > 0));
            if (mine)
                sm[(rr * Q + my_slot - (M::nD + M::n0)) * kLdsW + hidx] =
                    *(gp<const raw>)(rowp + (long long)my_q * plane_bytes + hcolb);
        };
        stage(w + 1, std::integral_constant<int, 1>{});
        if (w == 0) stage(0, std::integral_constant<int, 2>{});
        if (w == TH - 1) stage(TH + 1, std::integral_constant<int, 0>{});
        __syncthreads();

        const int y = y0 + w;
        // FP32 force sum with every lane of the wavefront (lanes past the
        // lattice take its last column)
        T Fx = 0, Fy = 0;
        if constexpr (MF) {
            if (K >= 0 && y < ny) {
                const float* row = (const float*)gtab + (size_t)y * 2 * J;
                const v4f acc = force_sum_global(row, row, bas + (size_t)min(x0 + lx, nx - 1) * J,
                                                 2 * (K + 1), fl);
                Fx = acc[0];
                Fy = acc[1];
            }
        }
        if (lx <= R && y < ny) {
            T f[Q];
            stream_interp<St, SM, mix_interp<S>>(
                [&](int q, int j, int i) -> T {
                    return (T)S::ld(&sm[M::srow(w + j, q) * kLdsW + 3 + lx + i]);
                },
                W, f);
            const SiteCtx<T> sctx{ginv, dt, K, gtab, eta_s};
            if constexpr (FORCED && F64) {
                if (K >= 0) {
                    const gp<const T> twx = (gp<const T>)twp;
                    force_cheb64(sctx, twx[2 * (x0 + lx)], twx[2 * (x0 + lx) + 1], y, Fx, Fy);
                }
            }
            update_site<S, St, FORCED>(f, sctx, Fx, Fy, (gp<char>)(dst + y * rowq_bytes), colb,
                                       A.d_flag);
        }
        __syncthreads();                     // before the next tile overwrites LDS
    }

    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        const int u0 = kTablesFirst ? (b < 0 ? b + extra : -1) : b - G;
        build_force_tables<T>(A, step, extra > 0 ? u0 : xcd + 8 * (b >> 3),
                              extra > 0 ? extra : 8 * nb);
    }
}

// ---------------------------------------------------------------------------
// Row-marching form of the same step.  A wavefront owns a strip of 64 columns
// and marches down a segment of rows [ya, yb).  Populations are loaded once per
// row, aligned, and kept in a rolling window of registers:
//   cur[q]  row y of every population,
//   up[.]   row y-1 of the populations pulled from the row above (c_y > 0),
//   dn[.]   row y+1 of the populations pulled from the row below (c_y < 0),
//   pre[q]  the next row in flight (y+1, or y+2 for the c_y < 0 ones).
// Horizontal neighbours come from the neighbouring lane (ds_bpermute); the edge
// lane takes the strip's halo column, fetched for all populations of a row by
// one gathered load (lane j holds the halo of the j-th population with
// c_x != 0).  The per-site arithmetic is the same update_site as the tile form,
// so both forms give bitwise identical results.  The new populations are
// written with non-temporal stores: this form serves lattices much larger than
// the caches, whose new state is not read again until the next launch.
// ---------------------------------------------------------------------------
template <class St>
struct MarchMap {
    static constexpr int Q = St::Q;
    static constexpr int cx(int q) { return St::dir[q].cx; }
    static constexpr int cy(int q) { return St::dir[q].cy; }
    static constexpr int count(int kind) {       // 0: c_y > 0, 1: c_y < 0
        int n = 0;
        for (int q = 0; q < Q; ++q) n += kind == 0 ? (cy(q) > 0) : (cy(q) < 0);
        return n;
    }
    static constexpr int nU = count(0);
    static constexpr int nD = count(1);
    static constexpr int uidx(int q) {
        int k = 0;
        for (int p = 0; p < q; ++p) k += cy(p) > 0;
        return k;
    }
    static constexpr int didx(int q) {
        int k = 0;
        for (int p = 0; p < q; ++p) k += cy(p) < 0;
        return k;
    }
    // halo lanes: populations with c_x != 0, those with c_y >= 0 first
    static constexpr int nHUZ() {
        int k = 0;
        for (int q = 0; q < Q; ++q) k += (cx(q) != 0 && cy(q) >= 0);
        return k;
    }
    static constexpr int hidx(int q) {
        int k = 0;
        if (cy(q) >= 0) {
            for (int p = 0; p < q; ++p) k += (cx(p) != 0 && cy(p) >= 0);
            return k;
        }
        k = nHUZ();
        for (int p = 0; p < q; ++p) k += (cx(p) != 0 && cy(p) < 0);
        return k;
    }
    static constexpr int nH() {
        int k = 0;
        for (int q = 0; q < Q; ++q) k += cx(q) != 0;
        return k;
    }
};

template <class T>
__device__ __forceinline__ T read_lane(T v, int lane) {
    if constexpr (std::is_same<T, double>::value) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffu), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    }
}

// v from the lane one below (C > 0) or one above (C < 0) by a DPP wave shift
// (a vector-ALU move instead of an LDS permute); the lane that has no source
// lane (0 or 63) takes edge.
template <int C, class T>
__device__ __forceinline__ T lane_shift(T v, T edge) {
    constexpr int ctrl = C > 0 ? 0x138 : 0x130;        // wave_shr:1 / wave_shl:1
    if constexpr (std::is_same<T, double>::value) {
        const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
        const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)(e & 0xffffffffu),
                                                   (int)(unsigned)(b & 0xffffffffu), ctrl, 0xf, 0xf,
                                                   false);
        const int hi = __builtin_amdgcn_update_dpp((int)(e >> 32), (int)(b >> 32), ctrl, 0xf, 0xf,
                                                   false);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v),
                                                          ctrl, 0xf, 0xf, false));
    }
}

template <class T>
__device__ __forceinline__ T write_lane(T old, T val, int lane) {
    return (int)threadIdx.x == lane ? val : old;
}

template <class S, class St, int SM, bool FORCED>
__global__ __launch_bounds__(256) void march_kernel(StepArgs A) {
    static_assert(SM != kStreamHalo2, "the row-marching form streams from the nearest rows only");
    constexpr bool UNIT = SM == kStreamUnit;
    using T = typename S::T;
    using raw = typename S::raw;
    using M = MarchMap<St>;
    constexpr int Q = St::Q;
    constexpr int NH = M::nH();
    constexpr bool F64 = std::is_same<T, double>::value;
    constexpr bool MF = FORCED && !F64;       // FP32 force sums on the matrix cores

    const int64_t step = A.d_step[0] + A.step_off;
    const int par = (int)((A.d_step[1] + A.launch_off) & 1);
    const int lane = threadIdx.x;
    const int wv = uni((int)threadIdx.y);   // one wavefront per row of the block

    // XCD-aware persistent schedule over groups of 4 consecutive strip
    // segments (one per wavefront of the block)
    const int G = A.tile_blocks;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int n_groups = (A.n_tiles + 3) >> 2;
    const int chunk = (n_groups + 7) >> 3;
    const int g_end = min(n_groups, (xcd + 1) * chunk);

    // The loop over groups is uniform over the block (the basis barriers).
    for (int grp = b < G ? xcd * chunk + (b >> 3) : g_end; grp < g_end; grp += nb) {
        const int u = grp * 4 + wv;
        const int r = A.tile_real ? uni((int)A.tile_real[u]) : 0;
        const RealDesc& Dsc = A.desc[r];
        const int nx = uni(Dsc.nx), ny = uni(Dsc.ny);
        MarchItem it;
        it.decode(u - uni(Dsc.wm[A.map].tile_begin), uni(Dsc.wm[A.map].tiles_x), ny,
                  uni(Dsc.wm[A.map].seglen));
        const int ya = it.ya, yb = it.yb;
        const int x0 = it.strip * kTileW;
        const int R = min(kTileW - 1, nx - 1 - x0);      // last active lane
        const int x = x0 + lane;
        const bool active = lane <= R;
        int K = -1, J = 0;
        if constexpr (FORCED) {
            K = uni(Dsc.K);
            if constexpr (MF) J = uni(Dsc.J);
        }
        if constexpr (MF) {
            // this strip's force basis, shared by the block's four wavefronts
            // (columns past the lattice take its last column's)
            __syncthreads();
            if (K >= 0)
                stage_basis(uni(Dsc.bas), J, kTileW, [&](int col) { return min(x0 + col, nx - 1); });
            __syncthreads();
        }
        if (!it.rows) continue;
        constexpr long long plane_bytes = kTileW * sizeof(raw);
        const long long rowq = (long long)uni(Dsc.pitch) * Q * (long long)sizeof(raw);
        const char* src = (const char*)uni(Dsc.buf[par]);
        char* dst = (char*)uni(Dsc.buf[par ^ 1]);
        InterpW<T> W;
        SiteCtx<T> sctx;
        if constexpr (F64) {
            W.set(uni(Dsc.a[0]), uni(Dsc.a[1]), uni(Dsc.a[2]));
            sctx.ginv = uni(Dsc.inv_tau);
            sctx.dt = uni(Dsc.dt);
        } else {
            W.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
            sctx.ginv = uni(Dsc.inv_tauf);
            sctx.dt = uni(Dsc.dtf);
        }
        sctx.K = K;
        sctx.eta_s = uni(Dsc.tau_mode);
        sctx.gtab = nullptr;
        T c1 = 0, s1 = 0;
        if constexpr (FORCED) {
            sctx.gtab = uni((const T*)Dsc.g[step & 3]);
            if constexpr (F64) {
                if (K >= 0 && active) {
                    const gp<const T> twx = (gp<const T>)uni((const T*)Dsc.twx);
                    c1 = twx[2 * x];
                    s1 = twx[2 * x + 1];
                }
            }
        }
        // FP32 forms: force sums on the vector ALU (basis in LDS)
        const float* gsf = nullptr;
        if constexpr (MF) gsf = (const float*)sctx.gtab;
        const int cols[1] = {lane};
        const uint32_t colb = col_bytes<raw>(x, Q);
        auto wrap = [&](int yy) { return yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy); };
        auto ld = [&](int q, int yy) -> T {
            const char* rowp = src + (long long)wrap(yy) * rowq + (long long)q * plane_bytes;
            return (T)S::ld((gp<const raw>)(rowp + colb));
        };
        // halo gather: lane j < NH holds the halo of the j-th population with c_x != 0,
        // row yy (c_y >= 0 populations) or yy + 1 (c_y < 0 populations)
        int my_q = 0, my_dy = 0;
        bool my_left = true;
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            if constexpr (M::cx(q) != 0) {
                if (lane == M::hidx(q)) {
                    my_q = q;
                    my_dy = M::cy(q) < 0 ? 1 : 0;
                    my_left = M::cx(q) > 0;
                }
            }
        });
        const int hcol = my_left ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + R + 1 == nx ? 0 : x0 + R + 1);
        auto gather = [&](int yy) -> T {
            T h = 0;
            if (lane < NH) {
                const char* p = src + (long long)wrap(yy + my_dy) * rowq +
                                (long long)my_q * plane_bytes + col_bytes<raw>(hcol, Q);
                h = (T)S::ld((gp<const raw>)p);
            }
            return h;
        };

        // prologue
        T cur[Q], pre[Q], up[M::nU], dn[M::nD];
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            cur[q] = ld(q, ya);
            if constexpr (M::cy(q) > 0) up[M::uidx(q)] = ld(q, ya - 1);
            if constexpr (M::cy(q) < 0) dn[M::didx(q)] = ld(q, ya + 1);
        });
        T hp = gather(ya - 1);
        T hc = gather(ya);
        T hn = 0;

        for (int y = ya; y < yb; ++y) {
            if (y + 1 < yb) {                    // next row in flight
                sfor<0, Q>([&](auto iq) {
                    constexpr int q = decltype(iq)::value;
                    pre[q] = ld(q, M::cy(q) < 0 ? y + 2 : y + 1);
                });
                hn = gather(y + 1);
            }
            // (b) stream: pull by linear interpolation
            T f[Q];
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                constexpr Dir d = St::dir[q];
                constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
                const T own = cur[q];
                T vert = own;
                if constexpr (d.cy > 0) vert = up[M::uidx(q)];
                if constexpr (d.cy < 0) vert = dn[M::didx(q)];
                if constexpr (d.cx == 0 && d.cy == 0) {
                    f[q] = own;
                } else if constexpr (d.cx == 0) {
                    if constexpr (UNIT && n == 1) f[q] = vert;
                    else f[q] = lerp<mix_interp<S>>(own, vert, W.a[n - 1]);
                } else {
                    // x-neighbour upstream: lane - 1 for c_x > 0, lane + 1 for c_x < 0,
                    // by a wave shift; the edge lane takes the halo column -- lane 0,
                    // or for c_x < 0 the last active lane R, through lane R + 1 when
                    // R < 63 (a ragged last strip) and as the shift's edge value
                    // when R = 63
                    constexpr int H = M::hidx(q);
                    auto shifted = [&](T v, T h) -> T {
                        if constexpr (d.cx > 0) return lane_shift<1>(v, h);
                        else return lane_shift<-1>(lane == R + 1 ? h : v, h);
                    };
                    const T h_own = read_lane(d.cy < 0 ? hp : hc, H);   // halo, row y
                    const T own_nb = shifted(own, h_own);
                    if constexpr (d.cy == 0) {
                        if constexpr (UNIT && n == 1) f[q] = own_nb;
                        else f[q] = lerp<mix_interp<S>>(own, own_nb, W.a[n - 1]);
                    } else {
                        // halo of the upstream row: y-1 (in hp) or y+1 (in hc)
                        const T h_vert = read_lane(d.cy > 0 ? hp : hc, H);
                        const T vert_nb = shifted(vert, h_vert);
                        f[q] = bilerp<mix_interp<S>>(own, own_nb, vert, vert_nb, W, n - 1);
                    }
                }
            });
            T Fx = 0, Fy = 0;
            if constexpr (MF) {
                if (K >= 0) {
                    float F[2];
                    force_sum_valu(gsf + (size_t)y * 2 * J, 2 * (K + 1), cols, kTileW, F);
                    Fx = F[0];
                    Fy = F[1];
                }
            } else if constexpr (FORCED) {
                force_cheb64(sctx, c1, s1, y, Fx, Fy);
            }
            if (active)
                update_site<S, St, FORCED, true>(f, sctx, Fx, Fy,
                                                 (gp<char>)(dst + (long long)y * rowq), colb,
                                                 A.d_flag);
            // roll the window
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                if constexpr (M::cy(q) > 0) {
                    up[M::uidx(q)] = cur[q];
                    cur[q] = pre[q];
                } else if constexpr (M::cy(q) < 0) {
                    cur[q] = dn[M::didx(q)];
                    dn[M::didx(q)] = pre[q];
                } else {
                    cur[q] = pre[q];
                }
            });
            hp = hc;
            hc = hn;
        }
    }

    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        build_force_tables<T>(A, step, extra > 0 ? b - G : xcd + 8 * (b >> 3),
                              extra > 0 ? extra : 8 * nb);
    }
}

// ---------------------------------------------------------------------------
// Paired row-marching form, for the 16-bit storage forms.  Every lane owns
// two adjacent columns of a 128-column strip, so each load and store moves an
// aligned 32-bit pair (256 bytes per wavefront instruction, two whole cache
// lines, as in the FP32 forms).  Needs even nx: the strip's last column is
// then always the high half of a pair.  With column A = 2 l (the low half)
// and column B = 2 l + 1 (the high half) of lane l:
//   c_x > 0: A pulls from the high half of lane l - 1, B from its low half;
//   c_x < 0: A pulls from its high half, B from the low half of lane l + 1;
// the lane exchanges are DPP wave shifts.  Lanes past the lattice's last
// column hold the periodically wrapped columns, so in a ragged last strip the
// last column's right neighbour (column 0) comes from the next lane; the
// strip's halo columns x0 - 1 and x0 + 128 enter as the DPP shift's value for
// the lane without a source lane (0 or 63): one gathered load per row (lane j
// holds the halo of the j-th population with c_x != 0), read out by
// v_readlane.
// The lane streams and updates column A, then column B, so one site's
// streamed populations are live at a time; column B's new populations go
// into the high halves of the words that hold column A's (S::pk_first /
// pk_second).  Both sites go through the same per-site update as every other
// form, so the results are bitwise identical.
// Stirring force: the sums of force_chunk (site.hpp) on the matrix cores,
// two chains (columns A and B) over the same coefficient registers and two
// rows at a time (outputs 0, 1: row y; 2, 3: row y + 1), in every other row
// iteration after its loads are issued, from coefficients loaded at the start
// of the iteration before, ahead of its population loads: a whole row
// iteration hides their latency, and waiting for them never waits for a
// population row.  The strip's basis sits in LDS as [J/4][A, B][lane] (16-byte reads
// without bank conflicts).
// Two wavefronts per SIMD: with three (at most 168 VGPRs) the forced kernel
// spills, and 8192^2 F16S ran 14 % slower.
// ---------------------------------------------------------------------------
template <class S, class St, int SM, bool FORCED>
__global__ __launch_bounds__(256, 2) void march_pair_kernel(StepArgs A) {
    static_assert(SM != kStreamHalo2, "the row-marching form streams from the nearest rows only");
    static_assert(sizeof(typename S::raw) == 2, "pairs of 16-bit populations");
    constexpr bool UNIT = SM == kStreamUnit;
    using T = typename S::T;
    using raw = typename S::raw;
    using M = MarchMap<St>;
    constexpr int Q = St::Q;
    constexpr int kW = 2 * kTileW;              // columns per strip
    constexpr int NH = M::nH();

    const int64_t step = A.d_step[0] + A.step_off;
    const int par = (int)((A.d_step[1] + A.launch_off) & 1);
    const int lane = threadIdx.x;
    const int wv = uni((int)threadIdx.y);
    ForceLane fl;
    fl.init(lane);

    const int G = A.tile_blocks;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int n_groups = (A.n_tiles + 3) >> 2;
    const int chunk = (n_groups + 7) >> 3;
    const int g_end = min(n_groups, (xcd + 1) * chunk);

    // x-neighbours: the pair of lane l - 1 (wave_shr:1) or l + 1 (wave_shl:1);
    // the lane without a source lane (0 or 63) takes edge
    auto from_left = [](uint32_t v, uint32_t edge) -> uint32_t {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xf, 0xf, false);
    };
    auto from_right = [](uint32_t v, uint32_t edge) -> uint32_t {
        return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xf, 0xf, false);
    };
    auto halo_bits = [](uint32_t h, int l) -> uint32_t {
        return (uint32_t)__builtin_amdgcn_readlane((int)h, l);
    };

    // The loop over groups is uniform over the block (the basis barriers).
    for (int grp = b < G ? xcd * chunk + (b >> 3) : g_end; grp < g_end; grp += nb) {
        const int u = grp * 4 + wv;
        const int r = A.tile_real ? uni((int)A.tile_real[u]) : 0;
        const RealDesc& Dsc = A.desc[r];
        const int nx = uni(Dsc.nx), ny = uni(Dsc.ny);
        MarchItem it;
        it.decode(u - uni(Dsc.wm[A.map].tile_begin), uni(Dsc.wm[A.map].tiles_x), ny,
                  uni(Dsc.wm[A.map].seglen));
        const int ya = it.ya, yb = it.yb;
        const int x0 = it.strip * kW;
        const int Rc = min(kW - 1, nx - 1 - x0);        // last column of the strip (odd)
        const int Lr = Rc >> 1;                         // its lane
        const int xa = x0 + 2 * lane;                   // this lane's columns xa, xa + 1
        const bool out_lane = lane <= Lr;
        const int xw = xa < nx ? xa : xa % nx;          // wrapped past the lattice
        int K = -1, J = 0;
        if constexpr (FORCED) {
            K = uni(Dsc.K);
            J = uni(Dsc.J);
            // this strip's force basis, shared by the block's four wavefronts:
            // position p < 64 holds column A of lane p, 64 + p column B
            // (columns past the lattice take its last column's)
            __syncthreads();
            if (K >= 0)
                stage_basis(uni(Dsc.bas), J, kW, [&](int pos) {
                    return min(x0 + (pos < kTileW ? 2 * pos : 2 * (pos - kTileW) + 1), nx - 1);
                });
            __syncthreads();
        }
        if (!it.rows) continue;
        constexpr long long plane_bytes = kTileW * sizeof(raw);
        const long long rowq = (long long)uni(Dsc.pitch) * Q * (long long)sizeof(raw);
        const char* src = (const char*)uni(Dsc.buf[par]);
        char* dst = (char*)uni(Dsc.buf[par ^ 1]);
        InterpW<T> W;
        SiteCtx<T> sctx;
        W.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
        sctx.ginv = uni(Dsc.inv_tauf);
        sctx.dt = uni(Dsc.dtf);
        sctx.K = K;
        sctx.eta_s = uni(Dsc.tau_mode);
        sctx.gtab = nullptr;
        if constexpr (FORCED) sctx.gtab = uni((const T*)Dsc.g[step & 3]);
        const uint32_t colb = col_bytes<raw>(xw, Q);
        auto wrap = [&](int yy) { return yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy); };
        // uniform row base (scalar registers), the lane's column as a 32-bit offset
        auto ld = [&](int q, int yy) -> uint32_t {
            const char* rowp = src + (long long)wrap(yy) * rowq + (long long)q * plane_bytes;
            return *(gp<const uint32_t>)(rowp + colb);
        };
        // halo gather of row yy: lane j < NH holds the 16 bits of the halo of
        // the j-th population with c_x != 0 at row yy -- column x0 - 1
        // (c_x > 0) or x0 + 128 (c_x < 0), wrapped (the other lanes read a
        // value they do not use)
        int my_q = 0;
        bool my_left = true;
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            if constexpr (M::cx(q) != 0) {
                if (lane == M::hidx(q)) {
                    my_q = q;
                    my_left = M::cx(q) > 0;
                }
            }
        });
        const int hcol = my_left ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + kW) % nx;
        const uint32_t hoff = (uint32_t)my_q * (uint32_t)plane_bytes + col_bytes<raw>(hcol, Q);
        auto gather = [&](int yy) -> uint32_t {
            const char* rowp = src + (long long)wrap(yy) * rowq;
            return *(gp<const uint16_t>)(rowp + hoff);
        };

        // force coefficients of rows yy, yy + 1 (the segment's last row for
        // rows past it): lane 4 t + m holds component m % 2 of term 16 c + t of
        // row yy (m < 2) or yy + 1 (m >= 2) in cf[c]; the first kPairCoefs
        // chunks (|kx| <= 47) are loaded ahead, further chunks where they are
        // used.  Rows yy and yy + 1 are adjacent in the table.
        constexpr int kPairCoefs = 6;
        const int jt = 2 * (K + 1);                     // terms that are not zero
        const int nch = J / kForceChunk;
        const float* gsf = (const float*)sctx.gtab;
        auto coef_row = [&](int yy) { return (gp<const float>)(gsf + (size_t)yy * 2 * J); };
        auto coef_off = [&](int yy) {      // this lane's offset from row yy (floats)
            return fl.off + (fl.hi && yy + 1 < yb ? 2u * (uint32_t)J : 0u);
        };
        float cf[kPairCoefs];
        auto load_row_coefs = [&](int yy) {
            const gp<const float> row = coef_row(yy);
            const uint32_t o = coef_off(yy);
#pragma unroll
            for (int c = 0; c < kPairCoefs; ++c)
                cf[c] = row[kForceChunk * 2 * min(c, nch - 1) + o];
        };
        v4f FA = {0.f, 0.f, 0.f, 0.f}, FB = {0.f, 0.f, 0.f, 0.f};
        // FA / FB = (Fx, Fy) of columns A / B at rows yy (0, 1) and yy + 1 (2, 3)
        auto force_rows = [&](int yy) {
            FA = {0.f, 0.f, 0.f, 0.f};
            FB = {0.f, 0.f, 0.f, 0.f};
            auto chunk = [&](int c, float a, auto all, int n) {
                v4f bA[4], bB[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    bA[i] = lds_basis[(4 * c + i) * kW + lane];
                    bB[i] = lds_basis[(4 * c + i) * kW + kTileW + lane];
                }
                force_chunk2<decltype(all)::value>(FA, FB, a, bA, bB, n);
            };
            // the chunk count and the last chunk's length pass through an
            // empty asm statement, so that the compiler compares them here
            // rather than keeping the comparisons' masks in scalar registers
            // across the row loop (which spilled them)
            int tail = force_tail(jt), nc = nch;
            asm volatile("" : "+s"(tail), "+s"(nc));
#pragma unroll
            for (int c = 0; c < kPairCoefs; ++c) {
                if (c + 1 < nc) chunk(c, cf[c], std::true_type{}, kForceChunk);
                else if (c + 1 == nc) chunk(c, cf[c], std::false_type{}, tail);
            }
            for (int c = kPairCoefs; c < nc; ++c)
                chunk(c, coef_row(yy)[kForceChunk * 2 * c + coef_off(yy)], std::false_type{},
                      c + 1 < nc ? kForceChunk : tail);
        };

        if constexpr (FORCED) {
            if (K >= 0) load_row_coefs(ya);
        }
        // The row window in three buffers whose roles rotate from row to row
        // (the row loop is unrolled three times, so the window never moves
        // between registers).  For a row y processed with buffers (X, Y, Z):
        //   c_y >= 0: X = row y - 1 (c_y > 0), Y = row y, Z <- row y + 1;
        //   c_y < 0:  X = row y, Y = row y + 1, Z <- row y + 2;
        // row y + 1 is processed with (Y, Z, X).
        uint32_t B0[Q], B1[Q], B2[Q];
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            if constexpr (M::cy(q) < 0) {
                B0[q] = ld(q, ya);
                B1[q] = ld(q, ya + 1);
            } else {
                if constexpr (M::cy(q) > 0) B0[q] = ld(q, ya - 1);
                B1[q] = ld(q, ya);
            }
        });
        // halo rows y - 1, y, y + 1 and (in flight) y + 2
        uint32_t hm = gather(ya - 1);
        uint32_t h0 = gather(ya);
        uint32_t h1 = gather(ya + 1);
        uint32_t h2 = 0;

        // Lane-shifted words of populations with c_x != 0 and c_y != 0 serve
        // two rows: the shift of row y is the streamed neighbour of row y and
        // the upstream neighbour of row y + 1 (c_y > 0), or that of row y - 1
        // and of row y (c_y < 0).  They rotate with the window: for row y with
        // shift buffers (SX, SY, SZ), SX holds the shift made one row earlier
        // and SY receives this row's.
        uint32_t T0[Q], T1[Q], T2[Q];
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            constexpr int H = M::hidx(q);
            if constexpr (M::cx(q) > 0 && M::cy(q) != 0)
                T0[q] = from_left(B0[q], halo_bits(M::cy(q) > 0 ? hm : h0, H) << 16);
            if constexpr (M::cx(q) < 0 && M::cy(q) != 0)
                T0[q] = from_right(B0[q], halo_bits(M::cy(q) > 0 ? hm : h0, H));
        });
        auto row = [&](int y, uint32_t (&X)[Q], uint32_t (&Y)[Q], uint32_t (&Z)[Q],
                       uint32_t (&SX)[Q], uint32_t (&SY)[Q], uint32_t (&SZ)[Q])
                       __attribute__((always_inline)) {
            const bool even = ((y - ya) & 1) == 0;
            // the coefficients of rows y + 1, y + 2, ahead of this row's loads
            if constexpr (FORCED) {
                if (K >= 0 && !even) load_row_coefs(min(y + 1, yb - 1));
            }
            // the next row in flight; issued in every iteration (past the
            // segment's rows it repeats its last, which is a cache hit), so
            // that the compiler's waits can leave these loads in flight
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                Z[q] = ld(q, M::cy(q) < 0 ? min(y + 2, yb) : min(y + 1, yb - 1));
            });
            h2 = gather(min(y + 2, yb));
            // the forces of rows y, y + 1 (coefficients loaded an iteration ago)
            if constexpr (FORCED) {
                if (K >= 0 && even) force_rows(y);
            }
            // column A.  Every lane streams and updates (the lane exchanges
            // need every lane's window); only the lanes on the lattice raise
            // the stability flag and store.
            T f[Q];
            typename S::pair_tmp tmp[Q];
            uint32_t outp[Q];
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                constexpr Dir d = St::dir[q];
                constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
                const uint32_t own = d.cy < 0 ? X[q] : Y[q];
                uint32_t vert = own;
                if constexpr (d.cy > 0) vert = X[q];
                if constexpr (d.cy < 0) vert = Y[q];
                const T oa = S::lo(own), va = S::lo(vert);
                if constexpr (d.cx == 0 && d.cy == 0) {
                    f[q] = oa;
                } else if constexpr (d.cx == 0) {
                    if constexpr (UNIT && n == 1) f[q] = va;
                    else f[q] = lerp<mix_interp<S>>(oa, va, W.a[n - 1]);
                } else {
                    // left neighbour of column A: lane l - 1's high half, for
                    // lane 0 the halo
                    constexpr int H = M::hidx(q);
                    T na;
                    if constexpr (d.cx > 0) {
                        if constexpr (d.cy > 0) na = S::hi(SY[q] = from_left(own, halo_bits(h0, H) << 16));
                        else if constexpr (d.cy < 0) na = S::hi(SX[q]);
                        else na = S::hi(from_left(own, halo_bits(h0, H) << 16));
                    } else {
                        na = S::hi(own);
                    }
                    if constexpr (d.cy == 0) {
                        if constexpr (UNIT && n == 1) f[q] = na;
                        else f[q] = lerp<mix_interp<S>>(oa, na, W.a[n - 1]);
                    } else {
                        // the upstream row's: y - 1 or y + 1
                        T vna;
                        if constexpr (d.cx > 0) {
                            if constexpr (d.cy > 0) vna = S::hi(SX[q]);
                            else vna = S::hi(SY[q] = from_left(vert, halo_bits(h1, H) << 16));
                        } else {
                            vna = S::hi(vert);
                        }
                        f[q] = bilerp<mix_interp<S>>(oa, na, va, vna, W, n - 1);
                    }
                }
            });
            update_site_fma<S, St, FORCED>(
                f, sctx, FA[0], FA[1],
                [&](auto qc, T a, T bb, T c) { tmp[decltype(qc)::value] = S::pk_first(a, bb, c); },
                A.d_flag, out_lane);
            // column B converts the window's halves anew: values kept from column
            // A's pass would stay live through A's update and cost registers
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (M::cy(i) != 0) asm volatile("" : "+v"(X[i]));
                asm volatile("" : "+v"(Y[i]));
            }
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                constexpr Dir d = St::dir[q];
                constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
                const uint32_t own = d.cy < 0 ? X[q] : Y[q];
                uint32_t vert = own;
                if constexpr (d.cy > 0) vert = X[q];
                if constexpr (d.cy < 0) vert = Y[q];
                const T ob = S::hi(own), vb = S::hi(vert);
                if constexpr (d.cx == 0 && d.cy == 0) {
                    f[q] = ob;
                } else if constexpr (d.cx == 0) {
                    if constexpr (UNIT && n == 1) f[q] = vb;
                    else f[q] = lerp<mix_interp<S>>(ob, vb, W.a[n - 1]);
                } else {
                    // right neighbour of column B: lane l + 1's low half, for
                    // lane 63 the halo
                    constexpr int H = M::hidx(q);
                    T nbv;
                    if constexpr (d.cx < 0) {
                        if constexpr (d.cy > 0) nbv = S::lo(SY[q] = from_right(own, halo_bits(h0, H)));
                        else if constexpr (d.cy < 0) nbv = S::lo(SX[q]);
                        else nbv = S::lo(from_right(own, halo_bits(h0, H)));
                    } else {
                        nbv = S::lo(own);
                    }
                    if constexpr (d.cy == 0) {
                        if constexpr (UNIT && n == 1) f[q] = nbv;
                        else f[q] = lerp<mix_interp<S>>(ob, nbv, W.a[n - 1]);
                    } else {
                        T vnb;
                        if constexpr (d.cx < 0) {
                            if constexpr (d.cy > 0) vnb = S::lo(SX[q]);
                            else vnb = S::lo(SY[q] = from_right(vert, halo_bits(h1, H)));
                        } else {
                            vnb = S::lo(vert);
                        }
                        f[q] = bilerp<mix_interp<S>>(ob, nbv, vb, vnb, W, n - 1);
                    }
                }
            });
            update_site_fma<S, St, FORCED>(
                f, sctx, FB[0], FB[1],
                [&](auto qc, T a, T bb, T c) {
                    constexpr int q = decltype(qc)::value;
                    outp[q] = S::pk_second(tmp[q], a, bb, c);
                },
                A.d_flag, out_lane);
            // row y + 1's forces
            FA[0] = FA[2];
            FA[1] = FA[3];
            FB[0] = FB[2];
            FB[1] = FB[3];
            // one 32-bit store per population and pair
            if (out_lane) {
                const gp<char> drow = (gp<char>)(dst + (long long)y * rowq);
                sfor<0, Q>([&](auto iq) {
                    constexpr int q = decltype(iq)::value;
                    __builtin_nontemporal_store(outp[q], (gp<uint32_t>)(drow + (long long)q * plane_bytes + colb));
                });
            }
            hm = h0;
            h0 = h1;
            h1 = h2;
        };
        for (int y = ya; y < yb; y += 3) {
            row(y, B0, B1, B2, T0, T1, T2);
            if (y + 1 >= yb) break;
            row(y + 1, B1, B2, B0, T1, T2, T0);
            if (y + 2 >= yb) break;
            row(y + 2, B2, B0, B1, T2, T0, T1);
        }
    }

    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        build_force_tables<T>(A, step, extra > 0 ? b - G : xcd + 8 * (b >> 3),
                              extra > 0 ? extra : 8 * nb);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch, row-marching.  A wavefront owns a strip of 62 output
// columns [x0, x0 + 62) and marches down its segment of rows [ya, yb) as in
// march_kernel, with 64 lanes on the columns x0 - 1 .. x0 + 62:
//   at step-n row r it streams the input (rolling window, lane exchange, halo
//   gathers for the columns x0 - 2 and x0 + 63) and applies update_site for
//   step s, keeping the new populations in registers (rounded to the storage
//   type, exactly as a one-step launch stores and reloads them);
//   it then streams step s + 1 at row r - 1 from the step-s rows r - 2, r - 1,
//   r held in registers (neighbours by lane exchange, no halo needed for
//   lanes 1..62) and stores rows [ya, yb) of step s + 2.
// Every population is read and written once per two steps; the step-s rows
// ya - 1 and yb and the two edge lanes are computed twice (by the
// neighbouring segment or strip).  The per-site arithmetic is the same
// update_site as every other form, so results are bitwise identical.
// ---------------------------------------------------------------------------
template <class S, class St, int SM, bool FORCED>
__global__ __launch_bounds__(512) void march2_kernel(StepArgs A) {
    static_assert(SM != kStreamHalo2, "the row-marching form streams from the nearest rows only");
    constexpr bool UNIT = SM == kStreamUnit;
    using T = typename S::T;
    using raw = typename S::raw;
    using M = MarchMap<St>;
    constexpr int Q = St::Q;
    constexpr int NH = M::nH();
    constexpr bool F64 = std::is_same<T, double>::value;
    constexpr bool MF = FORCED && !F64;       // FP32 force sums on the matrix cores
    constexpr int kOut = kTileW - 2;          // output columns per strip

    const int64_t step = A.d_step[0] + A.step_off;
    const int par = (int)((A.d_step[1] + A.launch_off) & 1);
    const int lane = threadIdx.x;
    const int wv = uni((int)threadIdx.y);
    ForceLane fl;
    fl.init(lane);

    const int G = A.tile_blocks;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int nb = (G - xcd + 7) >> 3;
    const int n_groups = (A.n_tiles + 7) >> 3;
    const int chunk = (n_groups + 7) >> 3;
    const int g_end = min(n_groups, (xcd + 1) * chunk);

    // The loop over groups is uniform over the block (the basis barriers).
    for (int grp = b < G ? xcd * chunk + (b >> 3) : g_end; grp < g_end; grp += nb) {
        const int u = grp * 8 + wv;
        const int r = A.tile_real ? uni((int)A.tile_real[u]) : 0;
        const RealDesc& Dsc = A.desc[r];
        const int nx = uni(Dsc.nx), ny = uni(Dsc.ny);
        MarchItem it;
        const int g = uni(Dsc.wm[A.map].group);
        it.decode_group(u - uni(Dsc.wm[A.map].tile_begin), uni(Dsc.wm[A.map].tiles_x), g, ny,
                        uni(Dsc.wm[A.map].seglen));
        const int ya = it.ya, yb = it.yb;
        const int x0 = it.strip * kOut;
        auto wrapx = [&](int v) { v %= nx; return v < 0 ? v + nx : v; };
        const int xl = wrapx(x0 - 1 + lane);     // column of this lane (both steps)
        const bool out_lane = lane >= 1 && lane <= kOut && x0 + lane - 1 < nx;
        int K = -1, J = 0;
        if constexpr (FORCED) {
            K = uni(Dsc.K);
            if constexpr (MF) J = uni(Dsc.J);
        }
        // this wavefront's strip's columns in the block's force basis (the
        // block's g strips side by side, 64 columns each)
        const int gs = it.strip - (it.strip / g) * g;
        const int bcol = lane + kTileW * gs;
        if constexpr (MF) {
            // the force basis of the block's strips (positions 64 s + col:
            // strip g p + s, column col; always four strips' positions, so
            // that the LDS stride is a constant), shared by its eight wavefronts
            const int xp = (it.strip - gs) * kOut;
            __syncthreads();                      // the previous strips' readers are done
            if (K >= 0)
                stage_basis(uni(Dsc.bas), J, 4 * kTileW, [&](int pos) {
                    return wrapx(xp + kOut * (pos >> 6) - 1 + (pos & 63));
                });
            __syncthreads();
        }
        if (!it.rows) continue;
        constexpr long long plane_bytes = kTileW * sizeof(raw);
        const long long rowq = (long long)uni(Dsc.pitch) * Q * (long long)sizeof(raw);
        const char* src = (const char*)uni(Dsc.buf[par]);
        char* dst = (char*)uni(Dsc.buf[par ^ 1]);
        InterpW<T> W;
        SiteCtx<T> c0, c1x;                       // contexts of steps s and s + 1
        if constexpr (F64) {
            W.set(uni(Dsc.a[0]), uni(Dsc.a[1]), uni(Dsc.a[2]));
            c0.ginv = uni(Dsc.inv_tau);
            c0.dt = uni(Dsc.dt);
        } else {
            W.set(uni(Dsc.af[0]), uni(Dsc.af[1]), uni(Dsc.af[2]));
            c0.ginv = uni(Dsc.inv_tauf);
            c0.dt = uni(Dsc.dtf);
        }
        c0.K = K;
        c0.eta_s = uni(Dsc.tau_mode);
        c0.gtab = nullptr;
        T cs = 0, sn = 0;
        if constexpr (FORCED) {
            c0.gtab = uni((const T*)Dsc.g[step & 3]);
            if constexpr (F64) {
                if (K >= 0) {
                    const gp<const T> twx = (gp<const T>)uni((const T*)Dsc.twx);
                    cs = twx[2 * xl];
                    sn = twx[2 * xl + 1];
                }
            }
        }
        c1x = c0;
        if constexpr (FORCED) c1x.gtab = uni((const T*)Dsc.g[(step + 1) & 3]);
        const uint32_t colb = col_bytes<raw>(xl, Q);
        auto wrap = [&](int yy) { return yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy); };
        auto ld = [&](int q, int yy) -> T {
            const char* rowp = src + (long long)wrap(yy) * rowq + (long long)q * plane_bytes;
            return (T)S::ld((gp<const raw>)(rowp + colb));
        };
        // halo gather of the input: lane j < NH holds the halo of the j-th
        // population with c_x != 0 (columns x0 - 2 and x0 + 63)
        int my_q = 0, my_dy = 0;
        bool my_left = true;
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            if constexpr (M::cx(q) != 0) {
                if (lane == M::hidx(q)) {
                    my_q = q;
                    my_dy = M::cy(q) < 0 ? 1 : 0;
                    my_left = M::cx(q) > 0;
                }
            }
        });
        const int hcol = my_left ? wrapx(x0 - 2) : wrapx(x0 + kTileW - 1);
        auto gather = [&](int yy) -> T {
            T h = 0;
            if (lane < NH) {
                const char* p = src + (long long)wrap(yy + my_dy) * rowq +
                                (long long)my_q * plane_bytes + col_bytes<raw>(hcol, Q);
                h = (T)S::ld((gp<const raw>)p);
            }
            return h;
        };

        // step-s rows r0 .. r1 feed the outputs ya .. yb - 1.  Iteration rr
        // first advances step s + 1 at row rr - 2 (from the step-s rows rr - 3,
        // rr - 2, rr - 1 computed earlier) and stores it, then computes step s
        // at row rr into registers: the stores are followed by a whole
        // site update before the next row's loads are needed.
        const int r0 = ya - 1, r1 = yb;
        // FP32 forms: the forces of iteration rr -- step s at row rr (outputs
        // 0, 1) and step s + 1 at row rr - 2 (outputs 2, 3) -- are summed at
        // the end of iteration rr - 1, from coefficients loaded at its start
        const int nch = J / kForceChunk;
        const float* gs0 = nullptr;
        const float* gs1 = nullptr;
        if constexpr (MF) {
            gs0 = (const float*)c0.gtab;
            gs1 = (const float*)c1x.gtab;
        }
        auto rowA = [&](int rr) { return gs0 + (size_t)wrap(min(rr, r1)) * 2 * J; };
        auto rowB = [&](int rr) { return gs1 + (size_t)max(ya, min(rr - 2, yb - 1)) * 2 * J; };
        v4f Fsum = {0.f, 0.f, 0.f, 0.f};
        float cf[kCoefRegs];
        if constexpr (MF) {
            if (K >= 0) {
                load_coefs(cf, rowA(r0), rowB(r0), nch, fl);
                Fsum = force_sum_lds(cf, rowA(r0), rowB(r0), 2 * (K + 1), bcol, 4 * kTileW, fl);
            }
        }
        T cur[Q], up[M::nU], dn[M::nD];           // input rows rr, rr - 1, rr + 1
        T nxt[Q];                                 // in flight: rr + 1 (c_y >= 0), rr + 2 (c_y < 0)
        T sa[M::nU], sb[Q], sp[Q];                // step-s rows rr - 3 (c_y > 0), rr - 2, rr - 1
        sfor<0, Q>([&](auto iq) {
            constexpr int q = decltype(iq)::value;
            cur[q] = ld(q, r0);
            if constexpr (M::cy(q) > 0) up[M::uidx(q)] = ld(q, r0 - 1);
            if constexpr (M::cy(q) < 0) dn[M::didx(q)] = ld(q, r0 + 1);
            nxt[q] = ld(q, M::cy(q) < 0 ? r0 + 2 : r0 + 1);
        });
        T hp = gather(r0 - 1);
        T hc = gather(r0);
        T hn = gather(r0 + 1);

        for (int rr = r0; rr <= r1 + 1; ++rr) {
            if constexpr (MF) {
                if (K >= 0) load_coefs(cf, rowA(rr + 1), rowB(rr + 1), nch, fl);
            }
            // step s + 1 at row rr - 2 from step-s rows rr - 3, rr - 2, rr - 1
            if (rr >= ya + 2) {
                T g[Q];
                sfor<0, Q>([&](auto iq) {
                    constexpr int q = decltype(iq)::value;
                    constexpr Dir d = St::dir[q];
                    constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
                    const T own = sb[q];
                    T vert = own;
                    if constexpr (d.cy > 0) vert = sa[M::uidx(q)];
                    if constexpr (d.cy < 0) vert = sp[q];
                    if constexpr (d.cx == 0 && d.cy == 0) {
                        g[q] = own;
                    } else if constexpr (d.cx == 0) {
                        if constexpr (UNIT && n == 1) g[q] = vert;
                        else g[q] = lerp<mix_interp<S>>(own, vert, W.a[n - 1]);
                    } else {
                        // lanes 1 .. 62 need no halo (edge lanes are not stored)
                        const T own_nb = lane_shift<d.cx>(own, own);
                        if constexpr (d.cy == 0) {
                            if constexpr (UNIT && n == 1) g[q] = own_nb;
                            else g[q] = lerp<mix_interp<S>>(own, own_nb, W.a[n - 1]);
                        } else {
                            const T vert_nb = lane_shift<d.cx>(vert, vert);
                            g[q] = bilerp<mix_interp<S>>(own, own_nb, vert, vert_nb, W, n - 1);
                        }
                    }
                });
                T Fx = 0, Fy = 0;
                if constexpr (MF) {
                    Fx = Fsum[2];
                    Fy = Fsum[3];
                } else if constexpr (FORCED) {
                    force_cheb64(c1x, cs, sn, rr - 2, Fx, Fy);
                }
                if (out_lane)
                    update_site<S, St, FORCED>(g, c1x, Fx, Fy,
                                               (gp<char>)(dst + (long long)(rr - 2) * rowq), colb,
                                               A.d_flag);
            }
            if (rr > r1) break;
            // step s at row rr, every lane
            T f[Q];
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                constexpr Dir d = St::dir[q];
                constexpr int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
                const T own = cur[q];
                T vert = own;
                if constexpr (d.cy > 0) vert = up[M::uidx(q)];
                if constexpr (d.cy < 0) vert = dn[M::didx(q)];
                if constexpr (d.cx == 0 && d.cy == 0) {
                    f[q] = own;
                } else if constexpr (d.cx == 0) {
                    if constexpr (UNIT && n == 1) f[q] = vert;
                    else f[q] = lerp<mix_interp<S>>(own, vert, W.a[n - 1]);
                } else {
                    // the edge lane (0 or 63) takes the strip's halo column
                    constexpr int H = M::hidx(q);
                    const T h_own = read_lane(d.cy < 0 ? hp : hc, H);
                    const T own_nb = lane_shift<d.cx>(own, h_own);
                    if constexpr (d.cy == 0) {
                        if constexpr (UNIT && n == 1) f[q] = own_nb;
                        else f[q] = lerp<mix_interp<S>>(own, own_nb, W.a[n - 1]);
                    } else {
                        const T h_vert = read_lane(d.cy > 0 ? hp : hc, H);
                        const T vert_nb = lane_shift<d.cx>(vert, h_vert);
                        f[q] = bilerp<mix_interp<S>>(own, own_nb, vert, vert_nb, W, n - 1);
                    }
                }
            });
            // The input window moves down one row now, from the row loaded one
            // iteration ago, and the row after it is loaded now.  Loads past
            // the rows the segment reads repeat its last rows (cache hits), so
            // that every iteration issues the same loads.
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                if constexpr (M::cy(q) > 0) {
                    up[M::uidx(q)] = cur[q];
                    cur[q] = nxt[q];
                } else if constexpr (M::cy(q) < 0) {
                    cur[q] = dn[M::didx(q)];
                    dn[M::didx(q)] = nxt[q];
                } else {
                    cur[q] = nxt[q];
                }
            });
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                nxt[q] = ld(q, M::cy(q) < 0 ? min(rr + 3, r1 + 1) : min(rr + 2, r1));
            });
            hp = hc;
            hc = hn;
            hn = gather(min(rr + 2, r1));
            T Fx = 0, Fy = 0;
            if constexpr (MF) {
                Fx = Fsum[0];
                Fy = Fsum[1];
            } else if constexpr (FORCED) {
                force_cheb64(c0, cs, sn, wrap(rr), Fx, Fy);
            }
            T fn[Q];
            update_site_to<S, St, FORCED>(
                f, c0, Fx, Fy,
                [&](auto qc, raw r) {              // the value a one-step launch stores
                    fn[decltype(qc)::value] = (T)S::ld(&r);
                },
                A.d_flag);
            // roll the step-s window
            sfor<0, Q>([&](auto iq) {
                constexpr int q = decltype(iq)::value;
                if constexpr (M::cy(q) > 0) sa[M::uidx(q)] = sb[q];
                sb[q] = sp[q];
                sp[q] = fn[q];
            });
            // the forces of the next iteration
            if constexpr (MF) {
                if (K >= 0) Fsum = force_sum_lds(cf, rowA(rr + 1), rowB(rr + 1), 2 * (K + 1), bcol, 4 * kTileW, fl);
            }
        }
    }

    if constexpr (FORCED) {
        const int extra = (int)gridDim.x - G;
        build_force_tables<T>(A, step, extra > 0 ? b - G : xcd + 8 * (b >> 3),
                              extra > 0 ? extra : 8 * nb);
    }
}

template <class St, int SM, bool FORCED>
static const void* kernel_ptr(int kind) {
    if constexpr (SM == kStreamHalo2) {
        // cfl > 1: tile form only
        return kind == kKernelTile ? (const void*)step_kernel<Store, St, SM, FORCED> : nullptr;
    } else {
        if (kind == kKernelMarch) return (const void*)march_kernel<Store, St, SM, FORCED>;
        if (kind == kKernelMarch2) return (const void*)march2_kernel<Store, St, SM, FORCED>;
        if (kind == kKernelStaged) return (const void*)staged_kernel<Store, St, SM, FORCED>;
        if (kind == kKernelMarchPair) {
            if constexpr (sizeof(typename Store::raw) == 2)
                return (const void*)march_pair_kernel<Store, St, SM, FORCED>;
            else
                return nullptr;
        }
        return (const void*)step_kernel<Store, St, SM, FORCED>;
    }
}

template <class St>
static const void* kernel_for(int kind, int smode, bool forced) {
    switch (smode) {
        case kStreamUnit:
            return forced ? kernel_ptr<St, kStreamUnit, true>(kind) : kernel_ptr<St, kStreamUnit, false>(kind);
        case kStreamHalo2:
            return forced ? kernel_ptr<St, kStreamHalo2, true>(kind) : kernel_ptr<St, kStreamHalo2, false>(kind);
        default:
            return forced ? kernel_ptr<St, kStreamGeneral, true>(kind) : kernel_ptr<St, kStreamGeneral, false>(kind);
    }
}

static const void* select_kernel(int kind, int stencil, int smode, bool forced) {
    if (stencil == RLBM_STENCIL_SPH26) return kernel_for<Sph26>(kind, smode, forced);
    if (stencil == RLBM_STENCIL_SPH26_ZFOLD) return kernel_for<Sph17>(kind, smode, forced);
    return kernel_for<Circ8>(kind, smode, forced);
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
    const void* k = select_kernel(L.kind, L.stencil, L.smode, L.forced);
    if (!k) return hipErrorInvalidDeviceFunction;
    StepArgs a = L.args;
    void* params[] = {&a};
    if (L.ev_start)
        return hipExtLaunchKernel(k, dim3(L.grid), dim3(kTileW, L.args.th), params, L.lds, L.stream,
                                  L.ev_start, L.ev_stop, 0);
    return hipLaunchKernel(k, dim3(L.grid), dim3(kTileW, L.args.th), params, L.lds, L.stream);
}

int RLBM_OCC_NAME(int kind, int stencil, int smode, bool forced, int th, size_t lds) {
    int blocks = 0;
    const void* k = select_kernel(kind, stencil, smode, forced);
    if (!k) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, kTileW * th, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace rlbm
