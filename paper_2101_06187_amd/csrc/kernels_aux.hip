// Auxiliary kernels: stirring-force table, step counter, initial state,
// population import/export, macroscopic fields, conserved sums, FFT passes
// and the shell-binned energy spectrum.
#include <algorithm>

#include "site.hpp"

namespace rlbm {

// ---------------------------------------------------------------------------
// force table of the current step (the step kernel builds the table of the
// step after it; this fills the first one after a state is set or loaded)
// ---------------------------------------------------------------------------
template <class T>
// the tables of steps d_step[0] + step_off and the step after it
__global__ void force_table_kernel(StepArgs A) {
    const int v = blockIdx.x;
    const int second = v >= A.n_gitems;
    const int u = second ? v - A.n_gitems : v;
    const int r = A.gitem_real ? uni((int)A.gitem_real[u]) : 0;
    const RealDesc& Dsc = A.desc[r];
    force_item<T>(Dsc, u - uni(Dsc.wm[A.map].gitem_begin), A.d_step[0] + A.step_off + second,
                  kTileW * A.th);
}

hipError_t launch_force_table(const StepArgs& a, bool fp32, hipStream_t s) {
    if (a.n_gitems <= 0) return hipSuccess;
    const dim3 grid(2 * a.n_gitems), block(kTileW, a.th);
    if (fp32) hipLaunchKernelGGL(force_table_kernel<float>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(force_table_kernel<double>, grid, block, 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// step counter and stability flag
// ---------------------------------------------------------------------------
__global__ void advance_kernel(int64_t* d_step, int64_t steps, int64_t flips) {
    if (threadIdx.x == 0) {
        volatile int64_t* p = d_step;
        p[0] = p[0] + steps;
        p[1] = p[1] + flips;
    }
}
__global__ void reset_kernel(int64_t* d_step, int64_t step, int64_t flips, int* d_flag) {
    if (threadIdx.x == 0) {
        volatile int64_t* p = d_step;
        volatile int* q = d_flag;
        p[0] = step;
        p[1] = flips;
        *q = 0;
    }
}
hipError_t launch_advance(int64_t* d_step, int64_t steps, int64_t flips, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, d_step, steps, flips);
    return hipGetLastError();
}
hipError_t launch_reset(int64_t* d_step, int64_t step, int64_t flips, int* d_flag, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, d_step, step, flips, d_flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initial state (Sec. III C step (a)): F = F_eq(eps, beta)
// ---------------------------------------------------------------------------
template <class S, class St>
__global__ void set_state_kernel(const RealDesc* desc, int r, const double* e,
                                 const double* ux, const double* uy, int parity) {
    const RealDesc& D = desc[r];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= D.nx) return;
    const int i = y * D.nx + x;
    double A0, B, C, gam;
    const double bx = ux[i], by = uy[i];
    eq_coeffs<St::D>(e[i], bx, by, A0, B, C, gam);
    typename S::raw* dst = (typename S::raw*)D.buf[parity];
    sfor<0, St::Q>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        constexpr double vx = dir_comp(St::dir[q], 0), vy = dir_comp(St::dir[q], 1);
        const double t = vx * bx + vy * by;
        const double F = fma(C, t * t, fma(B, t, A0));
        dst[pop_index(q, y, x, St::Q, D.pitch)] = S::from64(F - S::shift);
    });
}

template <class S, class St>
__global__ void set_pop_kernel(const RealDesc* desc, int r, const double* in, int parity) {
    const RealDesc& D = desc[r];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= D.nx) return;
    typename S::raw* dst = (typename S::raw*)D.buf[parity];
    for (int q = 0; q < St::Q; ++q)
        dst[pop_index(q, y, x, St::Q, D.pitch)] =
            S::from64(in[((long long)q * D.ny + y) * D.nx + x] - S::shift);
}

template <class S, class St>
__global__ void get_pop_kernel(const RealDesc* desc, int r, double* out, int parity) {
    const RealDesc& D = desc[r];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= D.nx) return;
    const typename S::raw* src = (const typename S::raw*)D.buf[parity];
    for (int q = 0; q < St::Q; ++q)
        out[((long long)q * D.ny + y) * D.nx + x] =
            S::to64(src[pop_index(q, y, x, St::Q, D.pitch)]) + S::shift;
}

// ---------------------------------------------------------------------------
// fields: stage (c) of the step in FP64 -- stream the current populations,
// form T^{mu nu}, solve the Landau frame.
// ---------------------------------------------------------------------------
template <class S, class St, int SM>
__global__ void fields_kernel(const RealDesc* desc, int r, int parity, double* e, double* ux,
                              double* uy, double* T, double2* z, int* d_flag) {
    const RealDesc& D = desc[r];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= D.nx) return;
    const int nx = D.nx, ny = D.ny;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const long long rowq = (long long)D.pitch * St::Q * (long long)sizeof(typename S::raw);
    const char* src = (const char*)uni(D.buf[parity]);
    double f[St::Q];
    if constexpr (SM == kStreamHalo2) {
        auto wrap = [](int v, int n) { return v < 0 ? (v + n < 0 ? v + 2 * n : v + n)
                                                    : (v >= n ? (v - n >= n ? v - 2 * n : v - n) : v); };
        const char* rows5[5];
        uint32_t cols5[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            rows5[j] = src + (long long)wrap(y + j - 2, ny) * rowq;
            cols5[j] = col_bytes<typename S::raw>(wrap(x + j - 2, nx), St::Q);
        }
        InterpW2<double> W2;
        W2.set(D.a[0], D.a[1], D.a[2]);
        stream_pull_h2<S, St, double>(rows5, cols5, W2, f);
    } else {
        const char* const rows[3] = {src + ym * rowq, src + y * rowq, src + yp * rowq};
        const uint32_t cols[3] = {col_bytes<typename S::raw>(xm, St::Q),
                                  col_bytes<typename S::raw>(x, St::Q),
                                  col_bytes<typename S::raw>(xp, St::Q)};
        InterpW<double> W;
        W.set(D.a[0], D.a[1], D.a[2]);
        stream_pull<S, St, SM, double>(rows, cols, W, f);
    }
    const Moments<double> m = moments<St, false>(f);
    const double sh = (double)S::shift;
    const double E = m.E + sh, Pxx = m.Pxx + sh / St::D, Pyy = m.Pyy + sh / St::D;
    double eps, bx, by;
    if (!landau64<St::D>(E, m.Jx, m.Jy, Pxx, m.Pxy, Pyy, eps, bx, by)) *d_flag = 1;
    const size_t i = (size_t)y * nx + x, n = (size_t)nx * ny;
    if (e) e[i] = eps;
    if (ux) ux[i] = bx;
    if (uy) uy[i] = by;
    if (T) {
        T[i] = E; T[n + i] = m.Jx; T[2 * n + i] = m.Jy;
        T[3 * n + i] = Pxx; T[4 * n + i] = m.Pxy; T[5 * n + i] = Pyy;
    }
    if (z) z[i] = make_double2(bx, by);
}

// ---------------------------------------------------------------------------
// conserved sums: sum over sites of T^00, T^0x, T^0y (stored populations),
// FP64, fixed reduction order (per-thread sequential, wave shuffle tree,
// block order, then one final block).
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* out) {
    __shared__ double sm[kRedThreads / 64][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) sm[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0;
            for (int k = 0; k < kRedThreads / 64; ++k) s += sm[k][c];
            out[c] = s;
        }
    }
}

int conserved_partials(int nx, int ny) {
    const long long n = (long long)nx * ny;
    long long b = (n + kRedThreads - 1) / kRedThreads;
    return (int)(b < 1024 ? b : 1024);
}

template <class S, class St>
__global__ void __launch_bounds__(kRedThreads)
conserved_kernel(const RealDesc* desc, int r, int parity, double* partials) {
    const RealDesc& D = desc[r];
    const long long n = (long long)D.nx * D.ny;
    const typename S::raw* src = (const typename S::raw*)D.buf[parity];
    double acc[3] = {0, 0, 0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const int y = (int)(i / D.nx), x = (int)(i - (long long)y * D.nx);
        double f[St::Q];
        for (int q = 0; q < St::Q; ++q)
            f[q] = S::to64(src[pop_index(q, y, x, St::Q, D.pitch)]);
        const Moments<double> m = moments<St, false>(f);
        acc[0] += m.E + (double)S::shift;
        acc[1] += m.Jx;
        acc[2] += m.Jy;
    }
    block_sum<3>(acc, partials + 3 * blockIdx.x);
}

__global__ void __launch_bounds__(kRedThreads)
final_sum_kernel(const double* partials, int n_partials, int nv, double* out) {
    for (int c = 0; c < nv; ++c) {
        double v[1] = {0};
        for (int i = threadIdx.x; i < n_partials; i += kRedThreads) v[0] += partials[i * nv + c];
        block_sum<1>(v, out + c);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FFT: one radix-2 Stockham pass over a batch of strided 1-D sequences.
// Pass with sub-transform size ns: a = in[j], c = in[j + n/2] * w^(k), k = j mod ns,
// w = exp(-2 pi i / (2 ns)); out[(j/ns) 2 ns + k] = a + c, out[... + ns] = a - c.
// After log2(n) passes the sequence is its DFT in natural order.
// ---------------------------------------------------------------------------
__global__ void fft_pass_kernel(const double2* in, double2* out, const double2* tw, int n,
                                int ns, int es, int bs, int batch) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int half = n >> 1;
    if (gid >= (long long)half * batch) return;
    int j, bi;
    if (es == 1) { bi = (int)(gid / half); j = (int)(gid - (long long)bi * half); }
    else { j = (int)(gid / batch); bi = (int)(gid - (long long)j * batch); }
    const int k = j % ns;
    const size_t base = (size_t)bi * bs;
    const double2 a = in[base + (size_t)j * es];
    const double2 c0 = in[base + (size_t)(j + half) * es];
    const double2 w = tw[(size_t)k * (n / (2 * ns))];
    const double2 c = make_double2(c0.x * w.x - c0.y * w.y, c0.x * w.y + c0.y * w.x);
    const int d = (j / ns) * 2 * ns + k;
    out[base + (size_t)d * es] = make_double2(a.x + c.x, a.y + c.y);
    out[base + (size_t)(d + ns) * es] = make_double2(a.x - c.x, a.y - c.y);
}

hipError_t launch_fft_pass(const double2* in, double2* out, const double2* tw, int n, int ns,
                           int es, int bs, int batch, hipStream_t s) {
    const long long work = (long long)(n / 2) * batch;
    hipLaunchKernelGGL(fft_pass_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       in, out, tw, n, ns, es, bs, batch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// driven-band filter (Sec. V).  Z = DFT(beta_x + i beta_y); a mode and its
// mirror -k have the same |k|, so zeroing Z(k) on the band removes the band
// from both components.  The inverse transform is done as a forward one of
// the conjugate: band_conj zeroes the band and conjugates the rest, the
// forward passes follow, unpack conjugates back, scales by 1/(nx ny), writes
// the two components and sums |beta| per block (fixed order).
// ---------------------------------------------------------------------------
__global__ void band_conj_kernel(double2* Z, int nx, int ny, double lo2, double hi2) {
    const long long n = (long long)nx * ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int iy = (int)(i / nx), ix = (int)(i - (long long)iy * nx);
        const long long kx = ix < nx / 2 ? ix : ix - nx;
        const long long ky = iy < ny / 2 ? iy : iy - ny;
        const double k2 = (double)(kx * kx + ky * ky);
        const double2 v = Z[i];
        Z[i] = (k2 >= lo2 && k2 <= hi2) ? make_double2(0.0, 0.0) : make_double2(v.x, -v.y);
    }
}

__global__ void __launch_bounds__(kRedThreads)
unpack_speed_kernel(const double2* W, int nx, int ny, double* ux, double* uy, double* partials) {
    const long long n = (long long)nx * ny;
    const double inv = 1.0 / ((double)nx * (double)ny);
    double acc[1] = {0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double2 v = W[i];
        const double bx = v.x * inv, by = -v.y * inv;
        if (ux) ux[i] = bx;
        if (uy) uy[i] = by;
        acc[0] += sqrt(bx * bx + by * by);
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

hipError_t launch_band_conj(double2* Z, int nx, int ny, double lo2, double hi2, hipStream_t s) {
    const long long n = (long long)nx * ny;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(band_conj_kernel, dim3(blocks), dim3(256), 0, s, Z, nx, ny, lo2, hi2);
    return hipGetLastError();
}

hipError_t launch_unpack_speed(const double2* W, int nx, int ny, double* ux, double* uy,
                               double* partials, int n_partials, double* out, hipStream_t s) {
    hipLaunchKernelGGL(unpack_speed_kernel, dim3(n_partials), dim3(kRedThreads), 0, s, W, nx, ny,
                       ux, uy, partials);
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n_partials,
                       1, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spectrum.  Z = DFT(beta_x + i beta_y).  For real beta the shell sum of
// 1/2 (|beta_hat_x|^2 + |beta_hat_y|^2) equals 1/2 sum_shell |Z(k)|^2 / (nx ny)^2
// (the shells are closed under k -> -k).  One wavefront per bin; lane l takes
// rows ky = ky_lo + l, ky_lo + l + 64, ...; mode k is in bin b iff
// (2b - 1)^2 <= 4 |k|^2 < (2b + 1)^2 (exact integer test; no ties).
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long isqrt_floor(long long v) {
    if (v <= 0) return 0;
    long long r = (long long)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

__device__ __forceinline__ double row_sum(const double2* Z, int nx, int ny, int ky, long long m_lo,
                                          long long m_hi) {
    const int iy = ky < 0 ? ky + ny : ky;
    double s = 0;
    for (long long m = m_lo; m <= m_hi; ++m) {
        // kx = +m (valid if m < nx/2) and kx = -m (valid if m > 0 and m <= nx/2)
        if (m < nx / 2) {
            const double2 v = Z[(size_t)iy * nx + m];
            s += v.x * v.x + v.y * v.y;
        }
        if (m > 0 && m <= nx / 2) {
            const double2 v = Z[(size_t)iy * nx + (nx - m)];
            s += v.x * v.x + v.y * v.y;
        }
    }
    return s;
}

__global__ void __launch_bounds__(64)
spectrum_bins_kernel(const double2* Z, int nx, int ny, int nbins, double* out) {
    const int b = blockIdx.x;
    if (b >= nbins) return;
    const long long lo2 = (long long)(2 * b - 1) * (2 * b - 1);   // for b >= 1
    const long long hi2 = (long long)(2 * b + 1) * (2 * b + 1);
    const int kyl = max(-(b + 1), -ny / 2), kyh = min(b + 1, ny / 2 - 1);
    double s = 0;
    for (int ky = kyl + (int)threadIdx.x; ky <= kyh; ky += 64) {
        const long long k2 = 4LL * ky * ky;
        if (k2 >= hi2) continue;
        // largest m with 4 (m^2 + ky^2) < hi2  <=>  4 m^2 <= hi2 - 1 - k2
        const long long m_hi = isqrt_floor((hi2 - 1 - k2) / 4);
        long long m_lo = 0;
        if (b >= 1 && lo2 > k2) {
            // smallest m with 4 m^2 >= lo2 - k2
            const long long need = lo2 - k2;
            m_lo = isqrt_floor((need + 3) / 4);
            while (4 * m_lo * m_lo < need) ++m_lo;
            while (m_lo > 0 && 4 * (m_lo - 1) * (m_lo - 1) >= need) --m_lo;
        }
        if (m_lo <= m_hi) s += row_sum(Z, nx, ny, ky, m_lo, min(m_hi, (long long)nx / 2));
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) {
        const double nn = (double)nx * (double)ny;
        out[b] = 0.5 * s / (nn * nn);
    }
}

int spectrum_partials(int nx, int ny) { return conserved_partials(nx, ny); }

__global__ void __launch_bounds__(kRedThreads)
enstrophy_kernel(const double2* Z, int nx, int ny, double* partials) {
    const long long n = (long long)nx * ny;
    const double inv = 1.0 / ((double)nx * (double)ny);
    double acc[1] = {0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const int iy = (int)(i / nx), ix = (int)(i - (long long)iy * nx);
        const int kx = ix < nx / 2 ? ix : ix - nx;
        const int ky = iy < ny / 2 ? iy : iy - ny;
        const double2 zk = Z[i];
        const double2 zr = Z[(size_t)((ny - iy) % ny) * nx + (nx - ix) % nx];
        // beta_hat_x = (Z(k) + conj Z(-k)) / 2,  beta_hat_y = -i (Z(k) - conj Z(-k)) / 2
        const double bxr = 0.5 * (zk.x + zr.x) * inv, bxi = 0.5 * (zk.y - zr.y) * inv;
        const double byr = 0.5 * (zk.y + zr.y) * inv, byi = -0.5 * (zk.x - zr.x) * inv;
        const double ax = 2.0 * M_PI * kx / nx, ay = 2.0 * M_PI * ky / ny;
        const double wr = ax * byr - ay * bxr, wi = ax * byi - ay * bxi;
        acc[0] += wr * wr + wi * wi;
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

hipError_t launch_spectrum_bins(const double2* Z, int nx, int ny, int nbins, double* out_bins,
                                double* partials, int n_partials, double* out_z, hipStream_t s) {
    hipLaunchKernelGGL(spectrum_bins_kernel, dim3(nbins), dim3(64), 0, s, Z, nx, ny, nbins,
                       out_bins);
    hipLaunchKernelGGL(enstrophy_kernel, dim3(n_partials), dim3(kRedThreads), 0, s, Z, nx, ny,
                       partials);
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n_partials,
                       1, out_z);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// dispatch on (storage, stencil)
// ---------------------------------------------------------------------------
template <template <class, class> class Fn, class... Args>
static hipError_t dispatch(int storage, int stencil, Args&&... args) {
    auto go = [&](auto s_tag) -> hipError_t {
        using S = decltype(s_tag);
        if (stencil == RLBM_STENCIL_SPH26) return Fn<S, Sph26>::run(args...);
        if (stencil == RLBM_STENCIL_SPH26_ZFOLD) return Fn<S, Sph17>::run(args...);
        return Fn<S, Circ8>::run(args...);
    };
    switch (storage) {
        case RLBM_F64: return go(StF64{});
        case RLBM_F32: return go(StF32{});
        case RLBM_F16S: return go(StF16S{});
        default: return go(StBF16S{});
    }
}

template <class S, class St>
struct SetStateFn {
    static hipError_t run(const RealDesc* d, int r, int nx, int ny, const double* e,
                          const double* ux, const double* uy, int parity, hipStream_t s) {
        hipLaunchKernelGGL((set_state_kernel<S, St>), dim3((nx + 127) / 128, ny), dim3(128), 0, s,
                           d, r, e, ux, uy, parity);
        return hipGetLastError();
    }
};
template <class S, class St>
struct SetPopFn {
    static hipError_t run(const RealDesc* d, int r, int nx, int ny, const double* in, int parity,
                          hipStream_t s) {
        hipLaunchKernelGGL((set_pop_kernel<S, St>), dim3((nx + 127) / 128, ny), dim3(128), 0, s, d,
                           r, in, parity);
        return hipGetLastError();
    }
};
template <class S, class St>
struct GetPopFn {
    static hipError_t run(const RealDesc* d, int r, int nx, int ny, double* out, int parity,
                          hipStream_t s) {
        hipLaunchKernelGGL((get_pop_kernel<S, St>), dim3((nx + 127) / 128, ny), dim3(128), 0, s, d,
                           r, out, parity);
        return hipGetLastError();
    }
};
template <class S, class St>
struct FieldsFn {
    static hipError_t run(const RealDesc* d, int r, int smode, int nx, int ny, int parity,
                          double* e, double* ux, double* uy, double* T, double2* z, int* flag,
                          hipStream_t s) {
        const dim3 g((nx + 127) / 128, ny), b(128);
        if (smode == kStreamUnit)
            hipLaunchKernelGGL((fields_kernel<S, St, kStreamUnit>), g, b, 0, s, d, r, parity, e, ux,
                               uy, T, z, flag);
        else if (smode == kStreamHalo2)
            hipLaunchKernelGGL((fields_kernel<S, St, kStreamHalo2>), g, b, 0, s, d, r, parity, e, ux,
                               uy, T, z, flag);
        else
            hipLaunchKernelGGL((fields_kernel<S, St, kStreamGeneral>), g, b, 0, s, d, r, parity, e,
                               ux, uy, T, z, flag);
        return hipGetLastError();
    }
};
template <class S, class St>
struct ConservedFn {
    static hipError_t run(const RealDesc* d, int r, int parity, double* partials, int np,
                          double* out3, hipStream_t s) {
        hipLaunchKernelGGL((conserved_kernel<S, St>), dim3(np), dim3(kRedThreads), 0, s, d, r,
                           parity, partials);
        hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, np, 3,
                           out3);
        return hipGetLastError();
    }
};

// ---------------------------------------------------------------------------
// z-mirror symmetry of imported populations (26-direction stencil): the
// one-layer lattice's states are even in v_z, and the step never forms the
// moments with one z index, so a state whose mirror pairs (a, b, c) /
// (a, b, -c) differ is outside what it computes.  Any differing pair (or a
// NaN) sets *word to 1; *word is cleared first by clear_word_kernel.
// ---------------------------------------------------------------------------
__global__ void clear_word_kernel(int* word) {
    if (threadIdx.x == 0) *(volatile int*)word = 0;
}

__global__ void mirror_check_kernel(const double* in, int nx, int ny, int* word) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx) return;
    const long long plane = (long long)nx * ny;
    const long long i = (long long)y * nx + x;
    bool bad = false;
    sfor<0, Sph26::Q>([&](auto iq) {
        constexpr int q = decltype(iq)::value;
        constexpr Dir d = Sph26::dir[q];
        if constexpr (d.cz < 0) {
            constexpr int m = mirror_of(q);
            bad |= !(in[q * plane + i] == in[m * plane + i]);
        }
    });
    if (bad) *(volatile int*)word = 1;
}

hipError_t launch_mirror_check(const double* in, int nx, int ny, int* word, hipStream_t s) {
    hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(64), 0, s, word);
    hipLaunchKernelGGL(mirror_check_kernel, dim3((nx + 127) / 128, ny), dim3(128), 0, s, in, nx,
                       ny, word);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy (measurement of the practical HBM ceiling): 16-byte elements,
// every block copies one contiguous chunk, four loads in flight per thread
// before the four stores.  n16 = bytes / 16.  (Measured on MI355X: at 1-7.5 GB
// per buffer 5.0-5.3 TB/s read + write, against 4.4-4.8 TB/s for the same
// loop striding over the whole grid; buffers that fit the 256 MB Infinity
// Cache copy faster.)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) stream_copy_kernel(const float4* __restrict__ src,
                                                          float4* __restrict__ dst, long long n16) {
    const long long per = (n16 + gridDim.x - 1) / gridDim.x;
    const long long b0 = (long long)blockIdx.x * per;
    const long long b1 = b0 + per < n16 ? b0 + per : n16;
    constexpr int kT = 256;
    for (long long i = b0 + threadIdx.x; i < b1; i += 4 * kT) {
        float4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * kT < b1) v[k] = src[i + k * kT];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * kT < b1) dst[i + k * kT] = v[k];
    }
}

hipError_t launch_stream_copy(const void* src, void* dst, long long n16, int blocks,
                              hipStream_t s) {
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, s, (const float4*)src,
                       (float4*)dst, n16);
    return hipGetLastError();
}

hipError_t launch_set_state(const RealDesc* d_desc, int r, int storage, int stencil, int nx,
                            int ny, const double* e, const double* ux, const double* uy,
                            int parity, hipStream_t s) {
    return dispatch<SetStateFn>(storage, stencil, d_desc, r, nx, ny, e, ux, uy, parity, s);
}
hipError_t launch_set_populations(const RealDesc* d_desc, int r, int storage, int stencil,
                                  int nx, int ny, const double* in, int parity, hipStream_t s) {
    return dispatch<SetPopFn>(storage, stencil, d_desc, r, nx, ny, in, parity, s);
}
hipError_t launch_get_populations(const RealDesc* d_desc, int r, int storage, int stencil,
                                  int nx, int ny, double* out, int parity, hipStream_t s) {
    return dispatch<GetPopFn>(storage, stencil, d_desc, r, nx, ny, out, parity, s);
}
hipError_t launch_fields(const RealDesc* d_desc, int r, int storage, int stencil, int smode,
                         int nx, int ny, int parity, double* e, double* ux, double* uy,
                         double* T, double2* z, int* d_flag, hipStream_t s) {
    return dispatch<FieldsFn>(storage, stencil, d_desc, r, smode, nx, ny, parity, e, ux, uy,
                              T, z, d_flag, s);
}
hipError_t launch_conserved(const RealDesc* d_desc, int r, int storage, int stencil, int nx,
                            int ny, int parity, double* partials, int n_partials, double* out3,
                            hipStream_t s) {
    (void)nx; (void)ny;
    return dispatch<ConservedFn>(storage, stencil, d_desc, r, parity, partials, n_partials, out3,
                                 s);
}

}  // namespace rlbm
