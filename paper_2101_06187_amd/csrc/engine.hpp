// Internal declarations shared by the device translation units and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rlbm.h"
#include "stencil.hpp"

namespace rlbm {

constexpr int kTileW = 64;            // sites per tile row = one wavefront
constexpr int kTableSlack = 32;       // compute-type values after the last row of a force table
constexpr int kForceTerms = 16;       // FP32 force terms are padded to a multiple of this

// Work decomposition of one lattice for one launch configuration.
struct WorkMap {
    int tiles_x, tiles_y;
    int tile_begin;               // first work item (tile or strip segment) of this lattice
    int seglen;                   // rows per strip segment (marching kernels)
    int gitem_begin;              // first force-table work item of this lattice
    int group;                    // two-step form: adjacent strips per block (1, 2 or 4)
};

// Per-lattice descriptor, resident in the workspace; every field is read
// once per tile and made wave-uniform.
struct RealDesc {
    void* buf[2];                 // population buffers; the current state is in
                                  // buf[flips & 1], flips = launches so far
    const void* twx;              // [nx][2] cos, sin of 2 pi x / nx (compute type)
    const void* twy;              // [ny][2] cos, sin of 2 pi y / ny (compute type)
    void* g[4];                   // force table of step s in g[s & 3]:
                                  //   FP64: [ny][K+1][4] = Px, Qx, Py, Qy;
                                  //   FP32: [ny][J][2], term 2k = (Px, Py),
                                  //   2k + 1 = (-Qx, -Qy), zero past 2 K + 1;
                                  //   then kTableSlack values that are never used
    const float* bas;             // FP32 forms: force basis [nx][J], term 2k =
                                  //   cos(2 pi k x / nx), 2k + 1 = sin(...)
    const int4* modes;            // (kx, ky, m, 0) grouped by |kx|
    const int* kptr;              // K+2 offsets into modes
    int nx, ny;
    int pitch;                    // nx rounded up to 64; see pop_index for the layout
    WorkMap wm[2];                // [0]: one-step launches, [1]: two-step launches
    int K;                        // largest |kx| of the driven modes; -1 unforced
    int J;                        // FP32 forms: force terms per row, 2 (K + 1)
                                  //   rounded up to kForceTerms (0 unforced)
    int n_modes;
    int realization;              // Philox counter word 2
    int tau_mode;                 // RLBM_TAU_CONSTANT or RLBM_TAU_ETA_S
    uint64_t seed;
    double amplitude;
    double inv_tau;               // 1 / tau
    double a[3];                  // interpolation weights cfl * |v| for 1, 2, 3
                                  // non-zero cube components
    double dt;                    // = cfl
    float af[3];
    float dtf;
    float inv_tauf;
    float amplitudef;
};

// A force-table work item covers one |kx| = k and 64 * th consecutive rows.
// A launch that advances steps [s, s + nsteps) reads the force tables of
// those steps and builds the tables of steps s + nsteps and s + nsteps + 1,
// so any sequence of one- and two-step launches finds its tables ready.
struct StepArgs {
    const RealDesc* desc;         // device array of descriptors
    const uint16_t* tile_real;    // tile -> lattice, NULL when there is one lattice
    const uint16_t* gitem_real;   // force item -> lattice, NULL when there is one lattice
    const int64_t* d_step;        // [0]: step counter, [1]: buffer flips (launches)
    int* d_flag;                  // stability flag
    int step_off;                 // this launch starts at step d_step[0] + step_off
    int launch_off;               // and reads buf[(d_step[1] + launch_off) & 1]
    int nsteps;                   // steps advanced by this launch (1 or 2)
    int map;                      // work map (RealDesc::wm) of this launch
    int n_tiles;
    int n_gitems;                 // force-table items of one table (0: unforced)
    int th;                       // wavefronts per block (tile height of the tile form)
    int tile_blocks;              // blocks [0, tile_blocks) walk the tiles; any further
                                  // blocks only build force tables
};

// Population layout in HBM ("row bricks").  Lattice row y is one contiguous
// block of Q * pitch elements (pitch = nx rounded up to 64) made of pitch / 64
// bricks; brick b holds columns [64 b, 64 b + 64): the 64 values of
// population 0, then those of population 1, and so on.  A wavefront's 64
// sites of one row thus read population q at a fixed offset q * 64 elements
// from the brick, which the load instructions carry as an immediate.
__host__ __device__ inline long long pop_index(int q, int y, int x, int Q, int pitch) {
    return (long long)y * Q * pitch + (long long)(x >> 6) * (Q * kTileW) + q * kTileW + (x & 63);
}
// byte offset of column x inside a row (same for every population)
template <class Raw>
__host__ __device__ inline uint32_t col_bytes(int x, int Q) {
    return (uint32_t)(((x >> 6) * (Q * kTileW) + (x & 63)) * (int)sizeof(Raw));
}

enum { kKernelTile = 0, kKernelMarch = 1, kKernelMarch2 = 2, kKernelStaged = 3, kKernelMarchPair = 4 };

// Stream modes: general cfl <= 1; cfl == 1 (axis populations move exactly
// one node); 1 < cfl <= 2 (sources up to two nodes upstream, tile form only).
enum { kStreamGeneral = 0, kStreamUnit = 1, kStreamHalo2 = 2 };

struct StepLaunch {
    StepArgs args;
    int kind;                     // kKernelTile or kKernelMarch
    int stencil;
    int smode;                    // kStreamGeneral / kStreamUnit / kStreamHalo2
    bool forced;
    int grid;                     // persistent blocks
    size_t lds = 0;               // dynamic LDS bytes per block
    hipStream_t stream;
    hipEvent_t ev_start = nullptr;  // optional: kernel start/stop timestamps
    hipEvent_t ev_stop = nullptr;
};

// Device translation units (one per storage form).
hipError_t launch_step_f64(const StepLaunch& L);
hipError_t launch_step_f32(const StepLaunch& L);
hipError_t launch_step_f16s(const StepLaunch& L);
hipError_t launch_step_bf16s(const StepLaunch& L);
// Resident blocks per CU of a step-kernel configuration (occupancy query).
int occ_f64(int kind, int stencil, int smode, bool forced, int th, size_t lds);
int occ_f32(int kind, int stencil, int smode, bool forced, int th, size_t lds);
int occ_f16s(int kind, int stencil, int smode, bool forced, int th, size_t lds);
int occ_bf16s(int kind, int stencil, int smode, bool forced, int th, size_t lds);

// Force table of the current step (kernels_aux.hip), for initial states.
hipError_t launch_force_table(const StepArgs& a, bool fp32, hipStream_t s);
hipError_t launch_advance(int64_t* d_step, int64_t steps, int64_t flips, hipStream_t s);
hipError_t launch_reset(int64_t* d_step, int64_t step, int64_t flips, int* d_flag, hipStream_t s);
hipError_t launch_set_state(const RealDesc* d_desc, int r, int storage, int stencil,
                            int nx, int ny, const double* e, const double* ux,
                            const double* uy, int parity, hipStream_t s);
hipError_t launch_set_populations(const RealDesc* d_desc, int r, int storage, int stencil,
                                  int nx, int ny, const double* in, int parity,
                                  hipStream_t s);
hipError_t launch_get_populations(const RealDesc* d_desc, int r, int storage, int stencil,
                                  int nx, int ny, double* out, int parity,
                                  hipStream_t s);
hipError_t launch_fields(const RealDesc* d_desc, int r, int storage, int stencil,
                         int smode, int nx, int ny, int parity, double* e,
                         double* ux, double* uy, double* T, double2* z,
                         int* d_flag, hipStream_t s);
hipError_t launch_mirror_check(const double* in, int nx, int ny, int* word, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, long long n16, int blocks,
                              hipStream_t s);
hipError_t launch_conserved(const RealDesc* d_desc, int r, int storage, int stencil,
                            int nx, int ny, int parity, double* partials,
                            int n_partials, double* out3, hipStream_t s);
int conserved_partials(int nx, int ny);
hipError_t launch_fft_pass(const double2* in, double2* out, const double2* tw, int n,
                           int ns, int elem_stride, int batch_stride, int batch,
                           hipStream_t s);
hipError_t launch_spectrum_bins(const double2* Z, int nx, int ny, int nbins,
                                double* out_bins, double* partials, int n_partials,
                                double* out_z, hipStream_t s);
int spectrum_partials(int nx, int ny);
hipError_t launch_band_conj(double2* Z, int nx, int ny, double lo2, double hi2, hipStream_t s);
hipError_t launch_unpack_speed(const double2* W, int nx, int ny, double* ux, double* uy,
                               double* partials, int n_partials, double* out, hipStream_t s);

}  // namespace rlbm
