// C ABI of the RLBM library: argument validation, workspace layout, forcing
// mode tables, launch sequencing (direct or through a captured HIP graph),
// diagnostics and checkpoints.  All device memory belongs to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "engine.hpp"

using namespace rlbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return fail(RLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int storage_bytes(int storage) {
    return storage == RLBM_F64 ? 8 : (storage == RLBM_F32 ? 4 : 2);
}
int stencil_q(int stencil) {
    return stencil == RLBM_STENCIL_SPH26 ? 26 : (stencil == RLBM_STENCIL_SPH26_ZFOLD ? 17 : 8);
}

struct ModeTable {
    std::vector<int4> modes;    // grouped by |kx|: (kx, ky, m, 0)
    std::vector<int> kptr;      // K + 2 entries
    int K = -1;
    int n = 0;
};

// Driven modes (Sec. V): integer (kx, ky), k_lo <= |k| <= k_hi, half plane
// ky > 0 or (ky == 0 and kx > 0), numbered in (ky, kx) lexicographic order.
int build_modes(const rlbm_lattice& lat, const rlbm_forcing* f, ModeTable& mt) {
    mt = ModeTable{};
    if (!f || f->amplitude == 0.0) return RLBM_OK;
    if (!(f->k_lo >= 0.0) || !(f->k_hi >= f->k_lo) || !std::isfinite(f->k_hi) ||
        !std::isfinite(f->amplitude))
        return fail(RLBM_EINVAL, "forcing shell must satisfy 0 <= k_lo <= k_hi, finite amplitude");
    const int kmax = (int)std::floor(f->k_hi) + 1;
    const double lo2 = f->k_lo * f->k_lo, hi2 = f->k_hi * f->k_hi;
    std::vector<int4> lex;
    for (int ky = 0; ky <= kmax; ++ky)
        for (int kx = -kmax; kx <= kmax; ++kx) {
            if (ky == 0 && kx <= 0) continue;
            const double k2 = (double)kx * kx + (double)ky * ky;
            if (k2 < lo2 || k2 > hi2) continue;
            if (2 * std::abs(kx) >= lat.nx || 2 * ky >= lat.ny)
                return fail(RLBM_EINVAL, "forcing shell reaches the Nyquist wave number");
            lex.push_back(make_int4(kx, ky, (int)lex.size(), 0));
        }
    mt.n = (int)lex.size();
    if (mt.n == 0) return RLBM_OK;
    for (const int4& m : lex) mt.K = std::max(mt.K, std::abs(m.x));
    mt.kptr.assign(mt.K + 2, 0);
    for (int k = 0; k <= mt.K; ++k) {
        mt.kptr[k] = (int)mt.modes.size();
        for (const int4& m : lex)
            if (std::abs(m.x) == k) mt.modes.push_back(m);
    }
    mt.kptr[mt.K + 1] = (int)mt.modes.size();
    return RLBM_OK;
}

// Terms of the FP32 force sum per row: 2 (K + 1) rounded up to kForceTerms
// (0 when the lattice is unforced).
int force_terms(const ModeTable& mt) {
    if (mt.n <= 0) return 0;
    return (2 * (mt.K + 1) + kForceTerms - 1) / kForceTerms * kForceTerms;
}

int validate_lattice(const rlbm_lattice* lat) {
    if (!lat) return fail(RLBM_EINVAL, "lattice is NULL");
    if (lat->nx < 2 || lat->ny < 2 || lat->nx > 65536 || lat->ny > 65536)
        return fail(RLBM_EINVAL, "lattice sides must be in [2, 65536]");
    if (!(lat->cfl > 0.0 && lat->cfl <= 2.0)) return fail(RLBM_EINVAL, "cfl must be in (0, 2]");
    return RLBM_OK;
}

int pitch_of(int nx) { return (nx + kTileW - 1) / kTileW * kTileW; }

// Workspace layout of one engine (descriptors, control words, reduction
// partials, tile map, then per lattice: two population buffers, twiddles,
// force tables, mode tables).
struct Layout {
    size_t ctl = 0, desc = 0, red = 0, tiles[2] = {0, 0}, gitems[2] = {0, 0}, total = 0;
    struct Per { size_t buf0, buf1, twx, twy, g[4], bas, modes, kptr; };
    std::vector<Per> per;
    int max_partials = 0;
};

int compute_layout(int n_real, const rlbm_lattice* lats, int stencil, int storage,
                   const std::vector<ModeTable>& mts, Layout& L) {
    const int Q = stencil_q(stencil), s = storage_bytes(storage);
    size_t off = 0;
    L.ctl = off; off = align_up(off + 64);
    L.desc = off; off = align_up(off + sizeof(RealDesc) * (size_t)n_real);
    const size_t cs = storage == RLBM_F64 ? sizeof(double) : sizeof(float);   // compute type
    int maxp = 1;
    long long tiles1 = 0, gitems1 = 0;
    for (int r = 0; r < n_real; ++r) {
        maxp = std::max(maxp, conserved_partials(lats[r].nx, lats[r].ny));
        // the narrowest work item: one row of a 62-column strip
        tiles1 += (long long)((lats[r].nx + kTileW - 3) / (kTileW - 2)) * lats[r].ny;
        gitems1 += (long long)(mts[r].K + 1) * ((lats[r].ny + kTileW - 1) / kTileW);
    }
    L.max_partials = maxp;
    L.red = off; off = align_up(off + sizeof(double) * (3 * (size_t)maxp + 8));
    for (int m = 0; m < 2; ++m) {
        L.tiles[m] = off;
        if (n_real > 1) off = align_up(off + sizeof(uint16_t) * (size_t)tiles1);
        L.gitems[m] = off;
        if (n_real > 1) off = align_up(off + sizeof(uint16_t) * (size_t)gitems1);
    }
    L.per.resize(n_real);
    for (int r = 0; r < n_real; ++r) {
        const size_t plane = (size_t)pitch_of(lats[r].nx) * lats[r].ny;
        auto& P = L.per[r];
        P.buf0 = off; off = align_up(off + plane * Q * s);
        P.buf1 = off; off = align_up(off + plane * Q * s);
        P.twx = off; off = align_up(off + cs * 2 * lats[r].nx);
        P.twy = off; off = align_up(off + cs * 2 * lats[r].ny);
        // force tables: FP64 [ny][K+1][4]; FP32 [ny][J][2] and the basis [nx][J]
        const int J = force_terms(mts[r]);
        const size_t g = storage == RLBM_F64 ? (size_t)lats[r].ny * (mts[r].K + 1) * 4 + kTableSlack
                                             : (size_t)lats[r].ny * 2 * J + kTableSlack;
        for (int k = 0; k < 4; ++k) { P.g[k] = off; off = align_up(off + cs * g); }
        P.bas = off;
        if (storage != RLBM_F64) off = align_up(off + sizeof(float) * (size_t)lats[r].nx * J);
        P.modes = off; off = align_up(off + sizeof(int4) * mts[r].modes.size());
        P.kptr = off; off = align_up(off + sizeof(int) * mts[r].kptr.size());
    }
    L.total = off;
    return RLBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// engine: one or more independent lattices advanced by one launch per step
// ---------------------------------------------------------------------------
struct Engine {
    // One launch configuration: kernel form and work decomposition.
    struct Cfg {
        int kind = kKernelTile;
        int th = 4;                 // wavefronts per block
        int seglen_req = 0, seglen = 0;
        int n_tiles = 0, n_gitems = 0, tile_blocks = 0, extra_blocks = 0, grid = 0;
        uint16_t* d_tiles = nullptr;     // tile -> lattice (ensembles)
        uint16_t* d_gitems = nullptr;    // force item -> lattice (ensembles)
    };

    int n_real = 0, stencil = 0, storage = 0, Q = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout lay;
    std::vector<rlbm_lattice> lats;
    std::vector<double> taus;
    std::vector<rlbm_forcing> frc;
    std::vector<ModeTable> mts;
    std::vector<RealDesc> hdesc;
    RealDesc* d_desc = nullptr;
    int64_t* d_step = nullptr;       // [0] steps, [1] buffer flips
    int* d_flag = nullptr;
    double* d_red = nullptr;
    int smode = kStreamUnit;         // stream mode of the step kernels (all lattices)
    bool any_forced = false;
    int cus = 0;
    int dev = 0;                     // device the engine was created on
    int maxJ = 0;                    // FP32 force terms per row, largest over the lattices
    Cfg cfg[2];                      // [0] one step per launch, [1] two steps per launch
    bool pairs = false;              // advance pairs of steps with cfg[1]
    bool kind_auto = true;           // until rlbm_set_kernel / rlbm_set_tile / autotune
    int64_t step = 0;
    int64_t flips = 0;               // launches since init; the state is in buf[flips & 1]
    int graph_chunk = 0;
    int graph_built_chunk = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap_stream = nullptr;

    ~Engine() { drop_graph(); if (cap_stream) (void)hipStreamDestroy(cap_stream); }

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_built_chunk = 0;
    }

    // Dynamic LDS of a launch: the marching forms of FP32 and 16-bit storage
    // keep their strip's force basis there (64 columns, 128 for the paired
    // form, J terms each).
    size_t lds_bytes(int kind) const {
        if (storage == RLBM_F64 || !any_forced) return 0;
        const size_t cols = kind == kKernelMarch2 ? 4 * kTileW
                            : kind == kKernelMarchPair ? 2 * kTileW
                            : kind == kKernelMarch ? kTileW : 0;
        return cols * (size_t)maxJ * sizeof(float);
    }
    // The marching forms hold at most kMaxMarchJ force terms per row in
    // registers and LDS (forcing shells with |kx| <= 63).
    static constexpr int kMaxMarchJ = 128;
    // the paired marching form keeps two adjacent columns per lane
    bool even_nx() const {
        for (const rlbm_lattice& l : lats)
            if (l.nx & 1) return false;
        return true;
    }
    bool kind_fits(int kind) const {
        return kind == kKernelTile || kind == kKernelStaged || storage == RLBM_F64 ||
               maxJ <= kMaxMarchJ;
    }

    int occupancy(int kind, int th) const {
        const size_t lds = lds_bytes(kind);
        switch (storage) {
            case RLBM_F64: return occ_f64(kind, stencil, smode, any_forced, th, lds);
            case RLBM_F32: return occ_f32(kind, stencil, smode, any_forced, th, lds);
            case RLBM_F16S: return occ_f16s(kind, stencil, smode, any_forced, th, lds);
            default: return occ_bf16s(kind, stencil, smode, any_forced, th, lds);
        }
    }

    long long wave_rows(int width) const {
        long long w = 0;
        for (int r = 0; r < n_real; ++r)
            w += (long long)((hdesc[r].nx + width - 1) / width) * hdesc[r].ny;
        return w;
    }

    // Default forms (measured on MI355X): the row-marching kernel when every
    // wavefront gets a strip segment of at least 8 rows (lattices far larger
    // than the caches) with FP32 or 16-bit storage, the tile kernel otherwise
    // (small lattices, FP64).  The best segment length depends on how the last
    // round of segments fills the chip (2048^2 FP32: 160 us at 32 rows, 186 us
    // at the default 22); rlbm_autotune searches it.  The two-step marching
    // kernel halves the memory traffic but holds both steps' rows in registers
    // (about 210 VGPRs, 2 wavefronts per SIMD); with short segments it is
    // 6-10 % faster per step than the one-step form for FP32 lattices far
    // larger than the caches and slower for 16-bit storage, the folded stencil
    // and cache-resident lattices.  It is used when requested or chosen by
    // rlbm_autotune.
    void choose_kind() {
        if (!kind_auto) return;
        Cfg& c = cfg[0];
        c.th = 4;
        const long long waves = (long long)cus * occupancy(kKernelMarch, 4) * 4;
        const bool long_segments = wave_rows(kTileW) >= 8 * std::max(1LL, waves);
        c.kind = (storage != RLBM_F64 && long_segments && smode != kStreamHalo2 &&
                  kind_fits(kKernelMarch)) ? kKernelMarch : kKernelTile;
        c.seglen_req = 0;
        pairs = false;
        cfg[1].kind = kKernelMarch2;
        cfg[1].th = 4;
        cfg[1].seglen_req = 0;
    }

    // work items (tiles of 64 x th sites, or strip segments of 64 columns --
    // 62 for the two-step kernel, 128 for the paired kernel -- x seglen rows),
    // their maps, the persistent grid
    int configure_map(int m) {
        Cfg& c = cfg[m];
        // 4 wavefronts per block (kStageTH), 8 for the two-step form
        if (c.kind != kKernelTile) c.th = c.kind == kKernelMarch2 ? 8 : 4;
        const int per_cu = occupancy(c.kind, c.th);
        const int slots = cus * per_cu;
        const int width = c.kind == kKernelMarch2 ? kTileW - 2
                          : (c.kind == kKernelMarchPair ? 2 * kTileW : kTileW);
        int seg = c.seglen_req;
        const bool tiled = c.kind == kKernelTile || c.kind == kKernelStaged;
        if (c.kind == kKernelMarch2 && seg <= 0) {
            // two-step form: short segments (measured, FP32: 2048^2 best at 12
            // rows, 153 us per step; 8192^2 at 16-32 rows; the one-segment-per-
            // wavefront length of the one-step forms, 35 and 547 rows, runs
            // 1.5-2x slower)
            seg = 12;
        } else if (!tiled && seg <= 0) {
            // about one strip segment per resident wavefront, at least 2 rows,
            // and no more segments than resident wavefronts (a few too many
            // would take a second round of the whole grid)
            const long long target = std::max(1LL, (long long)slots * 4);
            seg = (int)std::max(2LL, (wave_rows(width) + target - 1) / target);
            auto units = [&](int sl) {
                long long n = 0;
                for (int r = 0; r < n_real; ++r)
                    n += (long long)((hdesc[r].nx + width - 1) / width) *
                         (((hdesc[r].ny + sl - 1) / sl + 3) & ~3);
                return n;
            };
            while (units(seg) > target && seg < 65536) ++seg;
        }
        c.seglen = tiled ? c.th : seg;
        c.n_tiles = 0;
        c.n_gitems = 0;
        std::vector<uint16_t> map, gmap;
        const int rows = kTileW * c.th;               // rows per force-table item
        for (int r = 0; r < n_real; ++r) {
            RealDesc& d = hdesc[r];
            WorkMap& w = d.wm[m];
            w.tiles_x = (d.nx + width - 1) / width;
            w.seglen = c.seglen;
            w.tiles_y = (d.ny + w.seglen - 1) / w.seglen;
            // the marching forms number the segments of a strip consecutively,
            // padded to a multiple of the block's four wavefronts (which share
            // the strip's force basis)
            if (!tiled) w.tiles_y = (w.tiles_y + 3) & ~3;
            // the two-step form: blocks of g adjacent strips x 8 / g segments,
            // g = 4, 2 or 1: the largest whose padding (strips to a multiple of
            // g, segments to a multiple of 8 / g) adds at most 1/16 of the work
            // items, else the one that pads least (wide lattices: 4; the
            // ensemble's lattices of 2, 3 or 5 strips: 2 or 1)
            w.group = 1;
            int work = w.tiles_x * w.tiles_y;
            if (c.kind == kKernelMarch2) {
                const int segs = (d.ny + w.seglen - 1) / w.seglen;
                auto items = [&](int g) {
                    return (long long)8 * ((w.tiles_x + g - 1) / g) * ((segs + 8 / g - 1) / (8 / g));
                };
                const long long real = (long long)w.tiles_x * segs;
                long long best = -1;
                for (int g : {4, 2, 1}) {
                    if (16 * (items(g) - real) <= real) { w.group = g; best = -1; break; }
                    if (best < 0 || items(g) < best) { best = items(g); w.group = g; }
                }
                work = (int)items(w.group);
            }
            w.tile_begin = c.n_tiles;
            c.n_tiles += work;
            if (n_real > 1) map.insert(map.end(), (size_t)work, (uint16_t)r);
            w.gitem_begin = c.n_gitems;
            const int items = d.K >= 0 ? (d.K + 1) * ((d.ny + rows - 1) / rows) : 0;
            c.n_gitems += items;
            if (n_real > 1) gmap.insert(gmap.end(), (size_t)items, (uint16_t)r);
        }
        if (n_real > 1)
            HIPCHK(hipMemcpyAsync(c.d_tiles, map.data(), sizeof(uint16_t) * map.size(),
                                  hipMemcpyHostToDevice, stream));
        if (n_real > 1 && !gmap.empty())
            HIPCHK(hipMemcpyAsync(c.d_gitems, gmap.data(), sizeof(uint16_t) * gmap.size(),
                                  hipMemcpyHostToDevice, stream));
        const int groups = tiled ? c.n_tiles : (c.n_tiles + c.th - 1) / c.th;
        c.tile_blocks = std::max(8, std::min(groups, slots));
        // when the tiles leave resident slots free, build the next force tables
        // on extra blocks that run alongside the tiles
        c.extra_blocks = 0;
        if (any_forced && c.tile_blocks < slots) {
            c.extra_blocks = std::min(2 * c.n_gitems, slots - c.tile_blocks);
            // the tile and staged forms of FP32 and 16-bit storage put them
            // first: a multiple of 8 keeps every tile block on its XCD
            if (tiled && storage != RLBM_F64 && c.extra_blocks >= 8) c.extra_blocks &= ~7;
        }
        c.grid = c.tile_blocks + c.extra_blocks;
        return RLBM_OK;
    }

    int configure_tiles() {
        choose_kind();
        if (int rc = configure_map(0)) return rc;
        if (pairs)
            if (int rc = configure_map(1)) return rc;
        HIPCHK(hipMemcpyAsync(d_desc, hdesc.data(), sizeof(RealDesc) * n_real,
                              hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        drop_graph();
        return RLBM_OK;
    }

    // the main form: what rlbm_get_kernel reports and profile times
    int main_map() const { return pairs ? 1 : 0; }

    StepLaunch make_launch(int m, int step_off, int launch_off, hipStream_t s) const {
        const Cfg& c = cfg[m];
        StepLaunch L;
        L.kind = c.kind;
        L.args.desc = d_desc;
        L.args.tile_real = n_real > 1 ? c.d_tiles : nullptr;
        L.args.gitem_real = n_real > 1 ? c.d_gitems : nullptr;
        L.args.d_step = d_step;
        L.args.d_flag = d_flag;
        L.args.step_off = step_off;
        L.args.launch_off = launch_off;
        L.args.nsteps = c.kind == kKernelMarch2 ? 2 : 1;
        L.args.map = m;
        L.args.n_tiles = c.n_tiles;
        L.args.n_gitems = any_forced ? c.n_gitems : 0;
        L.args.th = c.th;
        L.args.tile_blocks = c.tile_blocks;
        L.stencil = stencil;
        L.smode = smode;
        L.forced = any_forced;
        L.grid = c.grid;
        L.lds = lds_bytes(c.kind);
        L.stream = s;
        return L;
    }

    hipError_t launch_step_kernel(StepLaunch& L) {
        switch (storage) {
            case RLBM_F64: return launch_step_f64(L);
            case RLBM_F32: return launch_step_f32(L);
            case RLBM_F16S: return launch_step_f16s(L);
            default: return launch_step_bf16s(L);
        }
    }

    hipError_t launch_on(StepLaunch& L, hipEvent_t before = nullptr, hipEvent_t after = nullptr) {
        L.ev_start = before;
        L.ev_stop = after;
        return launch_step_kernel(L);
    }

    // Launches for n steps on stream s (pairs first, then a single step);
    // returns the number of launches through *n_launches.
    hipError_t issue(int64_t n, hipStream_t s, int64_t* n_launches) {
        int64_t so = 0, lo = 0;
        if (pairs)
            for (; n - so >= 2; so += 2, ++lo) {
                StepLaunch L = make_launch(1, (int)so, (int)lo, s);
                if (hipError_t e = launch_on(L)) return e;
            }
        for (; so < n; ++so, ++lo) {
            StepLaunch L = make_launch(0, (int)so, (int)lo, s);
            if (hipError_t e = launch_on(L)) return e;
        }
        *n_launches = lo;
        return hipSuccess;
    }

    static int64_t launches_for(int64_t n, bool pairs_on) { return pairs_on ? n / 2 + n % 2 : n; }

    // n launches of the main form with events around every launch; mean
    // duration per launch in ms (a two-step launch advances two steps)
    int profile(int64_t n, double* avg_ms) {
        if (n < 1 || n > 100000) return fail(RLBM_EINVAL, "n must be in [1, 100000]");
        const int m = main_map();
        const int per = m == 1 ? 2 : 1;
        std::vector<hipEvent_t> ev(2 * n, nullptr);
        int rc = RLBM_OK;
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) { rc = fail(RLBM_EHIP, "hipEventCreate failed"); break; }
        for (int64_t i = 0; i < n && rc == RLBM_OK; ++i) {
            StepLaunch L = make_launch(m, (int)(i * per), (int)i, stream);
            if (launch_on(L, ev[2 * i], ev[2 * i + 1]) != hipSuccess)
                rc = fail(RLBM_EHIP, "launch failed while profiling");
        }
        if (rc == RLBM_OK && launch_advance(d_step, n * per, n, stream) != hipSuccess)
            rc = fail(RLBM_EHIP, "launch failed while profiling");
        if (rc == RLBM_OK) {
            step += n * per;
            flips += n;
        }
        double total = 0;
        if (rc == RLBM_OK && hipEventSynchronize(ev[2 * n - 1]) != hipSuccess)
            rc = fail(RLBM_EHIP, "hipEventSynchronize failed");
        for (int64_t i = 0; i < n && rc == RLBM_OK; ++i) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess)
                rc = fail(RLBM_EHIP, "hipEventElapsedTime failed");
            total += ms;
        }
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (rc == RLBM_OK && avg_ms) *avg_ms = total / (double)n;
        return rc;
    }

    // force tables of the current step and the next (after the populations
    // were set or loaded)
    int prime_force_table() {
        if (!any_forced) return RLBM_OK;
        StepLaunch L = make_launch(0, 0, 0, stream);
        HIPCHK(launch_force_table(L.args, storage != RLBM_F64, stream));
        return RLBM_OK;
    }

    int build_graph(int chunk) {
        drop_graph();
        if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        int64_t nl = 0;
        hipError_t err = issue(chunk, cap_stream, &nl);
        if (err == hipSuccess) err = launch_advance(d_step, chunk, nl, cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(RLBM_EHIP, std::string("graph capture failed: ") +
                                       hipGetErrorString(err != hipSuccess ? err : e2));
        }
        graph = g;
        HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        graph_built_chunk = chunk;
        return RLBM_OK;
    }

    int run(int64_t n) {
        if (n < 0) return fail(RLBM_EINVAL, "negative step count");
        int64_t done = 0;
        if (graph_chunk > 0 && n >= graph_chunk) {
            if (graph_built_chunk != graph_chunk) {
                int rc = build_graph(graph_chunk);
                if (rc != RLBM_OK) return rc;
            }
            const int64_t per_chunk = launches_for(graph_chunk, pairs);
            while (n - done >= graph_chunk) {
                HIPCHK(hipGraphLaunch(gexec, stream));
                done += graph_chunk;
                flips += per_chunk;
            }
        }
        const int64_t rest = n - done;
        if (rest > 0) {
            int64_t nl = 0;
            HIPCHK(issue(rest, stream, &nl));
            HIPCHK(launch_advance(d_step, rest, nl, stream));
            flips += nl;
        }
        step += n;
        return RLBM_OK;
    }

    int parity() const { return (int)(flips & 1); }
};

struct rlbm_ctx { Engine e; };
struct rlbm_batch { Engine e; };

namespace {

int engine_bytes(int n_real, const rlbm_lattice* lats, int stencil, int storage,
                 const rlbm_forcing* forcings, size_t* out) {
    if (!lats || !out) return fail(RLBM_EINVAL, "NULL argument");
    if (n_real < 1 || n_real > 65535) return fail(RLBM_EINVAL, "n_real must be in [1, 65535]");
    if (stencil != RLBM_STENCIL_SPH26 && stencil != RLBM_STENCIL_CIRC8 &&
        stencil != RLBM_STENCIL_SPH26_ZFOLD)
        return fail(RLBM_EINVAL, "unknown stencil");
    if (storage < RLBM_F64 || storage > RLBM_BF16S) return fail(RLBM_EINVAL, "unknown storage");
    std::vector<ModeTable> mts(n_real);
    for (int r = 0; r < n_real; ++r) {
        int rc = validate_lattice(&lats[r]);
        if (rc) return rc;
        const long long plane = (long long)pitch_of(lats[r].nx) * lats[r].ny;
        if (plane * (long long)storage_bytes(storage) >= (1LL << 31))
            return fail(RLBM_EINVAL, "one population plane must stay below 2 GiB");
        rc = build_modes(lats[r], forcings ? &forcings[r] : nullptr, mts[r]);
        if (rc) return rc;
    }
    Layout L;
    compute_layout(n_real, lats, stencil, storage, mts, L);
    *out = L.total;
    return RLBM_OK;
}

int engine_init(Engine& E, int n_real, const rlbm_lattice* lats, const double* taus, int stencil,
                const rlbm_forcing* forcings, int storage, void* ws, size_t ws_bytes,
                void* stream) {
    size_t need = 0;
    int rc = engine_bytes(n_real, lats, stencil, storage, forcings, &need);
    if (rc) return rc;
    if (!taus) return fail(RLBM_EINVAL, "tau is NULL");
    for (int r = 0; r < n_real; ++r)
        if (!(taus[r] > 0.5) || !std::isfinite(taus[r]))
            return fail(RLBM_EINVAL, "tau must be finite and > 0.5");
    if (!ws) return fail(RLBM_EINVAL, "workspace is NULL");
    if ((uintptr_t)ws % kAlign) return fail(RLBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(RLBM_ENOSPACE, "workspace too small");

    E.n_real = n_real;
    E.stencil = stencil;
    E.storage = storage;
    E.Q = stencil_q(stencil);
    E.stream = (hipStream_t)stream;
    E.ws = (char*)ws;
    E.lats.assign(lats, lats + n_real);
    E.taus.assign(taus, taus + n_real);
    E.frc.assign(n_real, rlbm_forcing{0.0, 0.0, 0.0, 0});
    if (forcings) E.frc.assign(forcings, forcings + n_real);
    E.mts.resize(n_real);
    for (int r = 0; r < n_real; ++r) build_modes(lats[r], &E.frc[r], E.mts[r]);
    compute_layout(n_real, lats, stencil, storage, E.mts, E.lay);

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&E.cus, hipDeviceAttributeMultiprocessorCount, dev));
    E.dev = dev;

    E.d_step = (int64_t*)(E.ws + E.lay.ctl);
    E.d_flag = (int*)(E.ws + E.lay.ctl + 16);
    E.d_desc = (RealDesc*)(E.ws + E.lay.desc);
    E.d_red = (double*)(E.ws + E.lay.red);
    for (int m = 0; m < 2; ++m) {
        E.cfg[m].d_tiles = (uint16_t*)(E.ws + E.lay.tiles[m]);
        E.cfg[m].d_gitems = (uint16_t*)(E.ws + E.lay.gitems[m]);
    }
    E.hdesc.assign(n_real, RealDesc{});
    E.smode = kStreamUnit;
    E.any_forced = false;
    const int s = storage_bytes(storage);
    for (int r = 0; r < n_real; ++r) {
        const auto& P = E.lay.per[r];
        const auto& lat = lats[r];
        RealDesc& d = E.hdesc[r];
        std::memset(&d, 0, sizeof(d));
        d.buf[0] = E.ws + P.buf0;
        d.buf[1] = E.ws + P.buf1;
        d.twx = E.ws + P.twx;
        d.twy = E.ws + P.twy;
        for (int k = 0; k < 4; ++k) d.g[k] = E.ws + P.g[k];
        d.bas = storage != RLBM_F64 ? (const float*)(E.ws + P.bas) : nullptr;
        d.J = storage != RLBM_F64 ? force_terms(E.mts[r]) : 0;
        E.maxJ = std::max(E.maxJ, d.J);
        d.modes = (const int4*)(E.ws + P.modes);
        d.kptr = (const int*)(E.ws + P.kptr);
        d.nx = lat.nx;
        d.ny = lat.ny;
        d.pitch = pitch_of(lat.nx);
        d.K = E.mts[r].n > 0 ? E.mts[r].K : -1;
        d.n_modes = E.mts[r].n;
        d.realization = r;
        d.seed = E.frc[r].seed;
        d.amplitude = E.frc[r].amplitude;
        d.amplitudef = (float)d.amplitude;
        d.inv_tau = 1.0 / taus[r];
        d.a[0] = lat.cfl;
        d.a[1] = lat.cfl * kInvSqrt2;
        d.a[2] = lat.cfl * kInvSqrt3;
        d.dt = lat.cfl;
        for (int i = 0; i < 3; ++i) d.af[i] = (float)d.a[i];
        d.dtf = (float)d.dt;
        d.inv_tauf = (float)d.inv_tau;
        if (lat.cfl > 1.0) E.smode = kStreamHalo2;
        else if (lat.cfl != 1.0 && E.smode == kStreamUnit) E.smode = kStreamGeneral;
        if (d.K >= 0) {
            E.any_forced = true;
        }
        (void)s;
    }
    // twiddles and mode tables (host -> workspace, synchronous at init)
    const bool f64 = storage == RLBM_F64;
    auto upload_tw = [&](size_t off, int n) -> int {
        std::vector<double> t64(2 * n);
        std::vector<float> t32(2 * n);
        for (int x = 0; x < n; ++x) {
            const double a = 2.0 * M_PI * (double)x / (double)n;
            t64[2 * x] = std::cos(a);
            t64[2 * x + 1] = std::sin(a);
            t32[2 * x] = (float)t64[2 * x];
            t32[2 * x + 1] = (float)t64[2 * x + 1];
        }
        if (f64)
            HIPCHK(hipMemcpyAsync(E.ws + off, t64.data(), sizeof(double) * t64.size(),
                                  hipMemcpyHostToDevice, E.stream));
        else
            HIPCHK(hipMemcpyAsync(E.ws + off, t32.data(), sizeof(float) * t32.size(),
                                  hipMemcpyHostToDevice, E.stream));
        HIPCHK(hipStreamSynchronize(E.stream));
        return RLBM_OK;
    };
    for (int r = 0; r < n_real; ++r) {
        const auto& P = E.lay.per[r];
        if (int rc2 = upload_tw(P.twx, lats[r].nx)) return rc2;
        if (int rc2 = upload_tw(P.twy, lats[r].ny)) return rc2;
        const int J = E.hdesc[r].J;
        if (!f64 && J > 0) {
            // FP32 force basis [nx][J]: term 2k = cos(2 pi k x / nx), 2k + 1 =
            // sin(...), rounded from FP64 at the exactly reduced angle (k x mod
            // nx); the terms past 2 K + 1 and the tables' padding terms are 0
            const int nx = lats[r].nx, K = E.mts[r].K;
            std::vector<float> bas((size_t)nx * J, 0.0f);
            for (int x = 0; x < nx; ++x)
                for (int k = 0; k <= K; ++k) {
                    const double a = 2.0 * M_PI * (double)(((long long)k * x) % nx) / (double)nx;
                    bas[(size_t)x * J + 2 * k] = (float)std::cos(a);
                    bas[(size_t)x * J + 2 * k + 1] = (float)std::sin(a);
                }
            HIPCHK(hipMemcpyAsync(E.ws + P.bas, bas.data(), sizeof(float) * bas.size(),
                                  hipMemcpyHostToDevice, E.stream));
            const size_t gbytes = sizeof(float) * ((size_t)lats[r].ny * 2 * J + kTableSlack);
            for (int k = 0; k < 4; ++k) HIPCHK(hipMemsetAsync(E.ws + P.g[k], 0, gbytes, E.stream));
            HIPCHK(hipStreamSynchronize(E.stream));
        }
        if (!E.mts[r].modes.empty()) {
            HIPCHK(hipMemcpyAsync(E.ws + P.modes, E.mts[r].modes.data(),
                                  sizeof(int4) * E.mts[r].modes.size(), hipMemcpyHostToDevice,
                                  E.stream));
            HIPCHK(hipMemcpyAsync(E.ws + P.kptr, E.mts[r].kptr.data(),
                                  sizeof(int) * E.mts[r].kptr.size(), hipMemcpyHostToDevice,
                                  E.stream));
        }
        HIPCHK(hipStreamSynchronize(E.stream));
    }
    HIPCHK(launch_reset(E.d_step, 0, E.flips, E.d_flag, E.stream));
    E.step = 0;
    return E.configure_tiles();
}

int check_ctx(const void* p) { return p ? RLBM_OK : fail(RLBM_EINVAL, "context is NULL"); }

int engine_set_relaxation(Engine& E, int mode) {
    if (mode != RLBM_TAU_CONSTANT && mode != RLBM_TAU_ETA_S)
        return fail(RLBM_EINVAL, "unknown relaxation mode");
    for (RealDesc& d : E.hdesc) d.tau_mode = mode;
    HIPCHK(hipMemcpyAsync(E.d_desc, E.hdesc.data(), sizeof(RealDesc) * E.n_real,
                          hipMemcpyHostToDevice, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
    return RLBM_OK;
}

int engine_set_state(Engine& E, int r, const double* d_e, const double* d_ux,
                     const double* d_uy, bool reset_step) {
    if (!d_e || !d_ux || !d_uy) return fail(RLBM_EINVAL, "NULL field pointer");
    if (reset_step) {
        HIPCHK(launch_reset(E.d_step, 0, E.flips, E.d_flag, E.stream));
        E.step = 0;
    }
    HIPCHK(launch_set_state(E.d_desc, r, E.storage, E.stencil, E.lats[r].nx, E.lats[r].ny, d_e,
                            d_ux, d_uy, E.parity(), E.stream));
    return E.prime_force_table();
}

int engine_fields(Engine& E, int r, double* d_e, double* d_ux, double* d_uy, double* d_T,
                  double2* z) {
    const double cfl = E.lats[r].cfl;
    const int fmode = cfl > 1.0 ? kStreamHalo2 : (cfl == 1.0 ? kStreamUnit : kStreamGeneral);
    HIPCHK(launch_fields(E.d_desc, r, E.storage, E.stencil, fmode, E.lats[r].nx,
                         E.lats[r].ny, E.parity(), d_e, d_ux, d_uy, d_T, z, E.d_flag, E.stream));
    return RLBM_OK;
}

int engine_check(Engine& E) {
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, E.d_flag, sizeof(int), hipMemcpyDeviceToHost, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
    return flag ? fail(RLBM_EUNSTABLE, "a site became unphysical") : RLBM_OK;
}

// checkpoint header
struct SaveHeader {
    char magic[8];
    int32_t version, stencil, storage, nx, ny, Q, tau_mode, reserved;
    int64_t step;
    double tau, cfl, amplitude, k_lo, k_hi;
    uint64_t seed;
};

}  // namespace

// ===========================================================================
// exported C ABI
// ===========================================================================
extern "C" {

const char* rlbm_status_string(int status) {
    switch (status) {
        case RLBM_OK: return "ok";
        case RLBM_EINVAL: return "invalid argument";
        case RLBM_ENOSPACE: return "workspace or buffer too small";
        case RLBM_EHIP: return "HIP runtime error";
        case RLBM_EUNSTABLE: return "unstable: a site became unphysical";
        case RLBM_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* rlbm_last_error(void) { return g_err.c_str(); }

int rlbm_stencil_info(int stencil, int32_t* h_q, double* h_v, double* h_w) {
    if (!h_q) return fail(RLBM_EINVAL, "h_q is NULL");
    auto fill = [&](auto st) {
        using St = decltype(st);
        *h_q = St::Q;
        for (int q = 0; q < St::Q; ++q) {
            for (int a = 0; a < 3; ++a)
                if (h_v) h_v[3 * q + a] = dir_comp(St::dir[q], a);
            if (h_w) {
                for (int c = 0; c < St::NC; ++c)
                    if (q >= St::cls[c].first &&
                        q < St::cls[c].first + St::cls[c].nplus + St::cls[c].nminus)
                        h_w[q] = St::cls[c].w;
            }
        }
    };
    if (stencil == RLBM_STENCIL_SPH26) fill(Sph26{});
    else if (stencil == RLBM_STENCIL_CIRC8) fill(Circ8{});
    else if (stencil == RLBM_STENCIL_SPH26_ZFOLD) fill(Sph17{});
    else return fail(RLBM_EINVAL, "unknown stencil");
    return RLBM_OK;
}

int rlbm_forcing_modes(const rlbm_lattice* lat, const rlbm_forcing* forcing, int32_t* h_kx,
                       int32_t* h_ky, int32_t cap, int32_t* h_n) {
    int rc = validate_lattice(lat);
    if (rc) return rc;
    if (!h_n || cap < 0 || (cap > 0 && (!h_kx || !h_ky))) return fail(RLBM_EINVAL, "bad output");
    ModeTable mt;
    rc = build_modes(*lat, forcing, mt);
    if (rc) return rc;
    // back to lexicographic order
    std::vector<int4> lex(mt.modes);
    std::sort(lex.begin(), lex.end(), [](const int4& a, const int4& b) { return a.z < b.z; });
    for (int i = 0; i < (int)lex.size() && i < cap; ++i) {
        h_kx[i] = lex[i].x;
        h_ky[i] = lex[i].y;
    }
    *h_n = mt.n;
    return RLBM_OK;
}

int rlbm_shell_modes(int32_t nx, int32_t ny, int32_t nbins, int64_t* h_counts) {
    if (nx < 1 || ny < 1 || nbins < 1 || !h_counts)
        return fail(RLBM_EINVAL, "bad shell-mode arguments");
    std::fill(h_counts, h_counts + nbins, (int64_t)0);
    const long long kx_lo = -(long long)(nx / 2), kx_hi = (long long)((nx - 1) / 2);
    const long long ky_lo = -(long long)(ny / 2), ky_hi = (long long)((ny - 1) / 2);
    const long long row = kx_hi - kx_lo + 1;
    for (long long ky = ky_lo; ky <= ky_hi; ++ky) {
        // round(|k|) <= b  <=>  4 |k|^2 < (2b + 1)^2  <=>  kx^2 <= b^2 + b - ky^2
        // (|k|^2 is an integer, so no |k| falls on a shell boundary).  Shells
        // below |ky| - 1 hold none of this row; r = floor(sqrt(b^2 + b - ky^2))
        // grows with b and is advanced, not recomputed.
        long long prev = 0, r = 0;
        for (long long b = std::max(0LL, std::llabs(ky) - 1); b < nbins && prev < row; ++b) {
            const long long m = b * b + b - ky * ky;
            if (m < 0) continue;
            while ((r + 1) * (r + 1) <= m) ++r;
            const long long c = std::max(0LL, std::min(r, kx_hi) - std::max(-r, kx_lo) + 1);
            h_counts[b] += c - prev;
            prev = c;
        }
    }
    return RLBM_OK;
}

int rlbm_spectrum_average(const double* h_samples, int32_t n_samples, int32_t nbins,
                          double* h_mean, double* h_err) {
    if (!h_samples || n_samples < 1 || nbins < 1 || !h_mean)
        return fail(RLBM_EINVAL, "bad spectrum-average arguments");
    const double inv = 1.0 / n_samples;
    for (int b = 0; b < nbins; ++b) {
        double s = 0;
        for (int i = 0; i < n_samples; ++i) s += h_samples[(size_t)i * nbins + b];
        const double m = s * inv;
        h_mean[b] = m;
        if (h_err) {
            double e = 0;
            for (int i = 0; i < n_samples; ++i) {
                const double v = h_samples[(size_t)i * nbins + b];
                e += std::sqrt(std::fabs(m * m - v * v));
            }
            h_err[b] = e * inv;
        }
    }
    return RLBM_OK;
}

int rlbm_workspace_bytes(const rlbm_lattice* lat, int stencil, int storage,
                         const rlbm_forcing* forcing, size_t* h_bytes) {
    return engine_bytes(1, lat, stencil, storage, forcing, h_bytes);
}

int rlbm_init(rlbm_ctx** out, const rlbm_lattice* lat, double tau, int stencil,
              const rlbm_forcing* forcing, int storage, void* d_workspace, size_t ws_bytes,
              void* hip_stream) {
    if (!out) return fail(RLBM_EINVAL, "out is NULL");
    *out = nullptr;
    rlbm_ctx* c = new (std::nothrow) rlbm_ctx();
    if (!c) return fail(RLBM_EINVAL, "out of host memory");
    int rc = engine_init(c->e, 1, lat, &tau, stencil, forcing, storage, d_workspace, ws_bytes,
                         hip_stream);
    if (rc) { delete c; return rc; }
    *out = c;
    return RLBM_OK;
}

int rlbm_set_state(rlbm_ctx* ctx, const double* d_e, const double* d_ux, const double* d_uy) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_set_state(ctx->e, 0, d_e, d_ux, d_uy, true);
}

int rlbm_step(rlbm_ctx* ctx, int64_t n) {
    if (int rc = check_ctx(ctx)) return rc;
    return ctx->e.run(n);
}

int rlbm_check(rlbm_ctx* ctx) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_check(ctx->e);
}

int rlbm_step_count(const rlbm_ctx* ctx, int64_t* h_steps) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!h_steps) return fail(RLBM_EINVAL, "NULL output");
    *h_steps = ctx->e.step;
    return RLBM_OK;
}

int rlbm_fields(rlbm_ctx* ctx, double* d_e, double* d_ux, double* d_uy, double* d_T) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_fields(ctx->e, 0, d_e, d_ux, d_uy, d_T, nullptr);
}

int rlbm_conserved(rlbm_ctx* ctx, double h_out[3]) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!h_out) return fail(RLBM_EINVAL, "NULL output");
    Engine& E = ctx->e;
    const int np = conserved_partials(E.lats[0].nx, E.lats[0].ny);
    double* out3 = E.d_red + 3 * (size_t)E.lay.max_partials;
    HIPCHK(launch_conserved(E.d_desc, 0, E.storage, E.stencil, E.lats[0].nx, E.lats[0].ny,
                            E.parity(), E.d_red, np, out3, E.stream));
    HIPCHK(hipMemcpyAsync(h_out, out3, 3 * sizeof(double), hipMemcpyDeviceToHost, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
    return RLBM_OK;
}

int rlbm_get_populations(rlbm_ctx* ctx, double* d_out) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!d_out) return fail(RLBM_EINVAL, "NULL output");
    Engine& E = ctx->e;
    HIPCHK(launch_get_populations(E.d_desc, 0, E.storage, E.stencil, E.lats[0].nx, E.lats[0].ny, d_out,
                                  E.parity(), E.stream));
    return RLBM_OK;
}

int rlbm_set_populations(rlbm_ctx* ctx, const double* d_in) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!d_in) return fail(RLBM_EINVAL, "NULL input");
    Engine& E = ctx->e;
    if (E.stencil == RLBM_STENCIL_SPH26) {
        // the 26-direction step assumes z-mirror symmetric states
        int* word = (int*)(E.ws + E.lay.ctl + 24);
        HIPCHK(launch_mirror_check(d_in, E.lats[0].nx, E.lats[0].ny, word, E.stream));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, word, sizeof(int), hipMemcpyDeviceToHost, E.stream));
        HIPCHK(hipStreamSynchronize(E.stream));
        if (bad)
            return fail(RLBM_EINVAL, "populations are not z-mirror symmetric: F(a, b, c) must "
                                     "equal F(a, b, -c) for every direction and site");
    }
    HIPCHK(launch_reset(E.d_step, 0, E.flips, E.d_flag, E.stream));
    E.step = 0;
    HIPCHK(launch_set_populations(E.d_desc, 0, E.storage, E.stencil, E.lats[0].nx, E.lats[0].ny, d_in,
                                  E.parity(), E.stream));
    return E.prime_force_table();
}

int rlbm_stream_copy(const void* d_src, void* d_dst, size_t bytes, int32_t reps,
                     void* hip_stream, double* h_ms) {
    if (!d_src || !d_dst || !h_ms) return fail(RLBM_EINVAL, "NULL pointer");
    if (bytes == 0 || bytes % 16 || (uintptr_t)d_src % 16 || (uintptr_t)d_dst % 16)
        return fail(RLBM_EINVAL, "bytes and both pointers must be non-zero multiples of 16");
    if (reps < 1) return fail(RLBM_EINVAL, "reps must be >= 1");
    const char* a = (const char*)d_src;
    const char* b = (const char*)d_dst;
    if (a < b + bytes && b < a + bytes) return fail(RLBM_EINVAL, "buffers overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const long long n16 = (long long)(bytes / 16);
    const int blocks = std::max(1, cus * 8);
    HIPCHK(launch_stream_copy(d_src, d_dst, n16, blocks, s));     // warm-up
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RLBM_EHIP, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, s);
    for (int i = 0; i < reps && err == hipSuccess; ++i) err = launch_stream_copy(d_src, d_dst, n16, blocks, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(RLBM_EHIP, std::string("stream copy: ") + hipGetErrorString(err));
    *h_ms = (double)ms / reps;
    return RLBM_OK;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Forward 2-D DFT by radix-2 Stockham passes, ping-ponging between a and b
// (rows with the x twiddles at sc + otx, then columns with sc + oty); returns
// the buffer holding the result, or NULL if a launch failed.
static double2* fft2_forward(Engine& E, char* sc, double2* a, double2* b, size_t otx,
                             size_t oty) {
    const int nx = E.lats[0].nx, ny = E.lats[0].ny;
    for (int ns = 1; ns < nx; ns *= 2) {   // rows (x)
        if (launch_fft_pass(a, b, (const double2*)(sc + otx), nx, ns, 1, nx, ny, E.stream) != hipSuccess)
            return nullptr;
        std::swap(a, b);
    }
    for (int ns = 1; ns < ny; ns *= 2) {   // columns (y)
        if (launch_fft_pass(a, b, (const double2*)(sc + oty), ny, ns, nx, 1, nx, E.stream) != hipSuccess)
            return nullptr;
        std::swap(a, b);
    }
    return a;
}

static size_t spectrum_layout(int nx, int ny, size_t* o_z2, size_t* o_twx, size_t* o_twy,
                              size_t* o_bins, size_t* o_part, size_t* o_out, int* max_bins) {
    const size_t n = (size_t)nx * ny;
    *max_bins = (int)std::ceil(std::sqrt((double)nx * nx / 4.0 + (double)ny * ny / 4.0)) + 2;
    size_t off = align_up(sizeof(double2) * n);
    *o_z2 = off; off = align_up(off + sizeof(double2) * n);
    *o_twx = off; off = align_up(off + sizeof(double2) * (nx / 2 + 1));
    *o_twy = off; off = align_up(off + sizeof(double2) * (ny / 2 + 1));
    *o_bins = off; off = align_up(off + sizeof(double) * (*max_bins));
    *o_part = off; off = align_up(off + sizeof(double) * spectrum_partials(nx, ny));
    *o_out = off; off = align_up(off + sizeof(double) * 8);
    return off;
}

int rlbm_spectrum_scratch_bytes(const rlbm_ctx* ctx, size_t* h_bytes) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!h_bytes) return fail(RLBM_EINVAL, "NULL output");
    size_t a, b, c, d, e, f;
    int mb;
    *h_bytes = spectrum_layout(ctx->e.lats[0].nx, ctx->e.lats[0].ny, &a, &b, &c, &d, &e, &f, &mb);
    return RLBM_OK;
}

// Forward 2-D DFT of beta_x + i beta_y of the current fields into the
// spectrum scratch; *out points at the transform (one of the two halves).
static int spectrum_transform(Engine& E, void* d_scratch, size_t scratch_bytes, double2** out,
                              int* max_bins) {
    const int nx = E.lats[0].nx, ny = E.lats[0].ny;
    if (!is_pow2(nx) || !is_pow2(ny))
        return fail(RLBM_EUNSUPPORTED, "the spectrum needs power-of-two lattice sides");
    if (!d_scratch) return fail(RLBM_EINVAL, "NULL scratch");
    size_t oz2, otx, oty, obins, opart, oout;
    const size_t need = spectrum_layout(nx, ny, &oz2, &otx, &oty, &obins, &opart, &oout, max_bins);
    if (scratch_bytes < need) return fail(RLBM_ENOSPACE, "spectrum scratch too small");
    if ((uintptr_t)d_scratch % kAlign) return fail(RLBM_EINVAL, "scratch must be 256-byte aligned");
    char* sc = (char*)d_scratch;
    std::vector<double2> twx(nx / 2 + 1), twy(ny / 2 + 1);
    for (int m = 0; m < nx / 2; ++m)
        twx[m] = make_double2(std::cos(2.0 * M_PI * m / nx), -std::sin(2.0 * M_PI * m / nx));
    for (int m = 0; m < ny / 2; ++m)
        twy[m] = make_double2(std::cos(2.0 * M_PI * m / ny), -std::sin(2.0 * M_PI * m / ny));
    HIPCHK(hipMemcpyAsync(sc + otx, twx.data(), sizeof(double2) * twx.size(),
                          hipMemcpyHostToDevice, E.stream));
    HIPCHK(hipMemcpyAsync(sc + oty, twy.data(), sizeof(double2) * twy.size(),
                          hipMemcpyHostToDevice, E.stream));
    double2* z = (double2*)sc;
    if (int rc = engine_fields(E, 0, nullptr, nullptr, nullptr, nullptr, z)) return rc;
    *out = fft2_forward(E, sc, z, (double2*)(sc + oz2), otx, oty);
    if (!*out) return fail(RLBM_EHIP, "FFT pass launch failed");
    return RLBM_OK;
}

int rlbm_spectrum(rlbm_ctx* ctx, void* d_scratch, size_t scratch_bytes, double* h_Ek,
                  int32_t nbins, double* h_enstrophy) {
    if (int rc = check_ctx(ctx)) return rc;
    Engine& E = ctx->e;
    if (!h_Ek || nbins < 1) return fail(RLBM_EINVAL, "bad spectrum arguments");
    const int nx = E.lats[0].nx, ny = E.lats[0].ny;
    double2* a = nullptr;
    int max_bins = 0;
    if (int rc = spectrum_transform(E, d_scratch, scratch_bytes, &a, &max_bins)) return rc;
    size_t oz2, otx, oty, obins, opart, oout;
    spectrum_layout(nx, ny, &oz2, &otx, &oty, &obins, &opart, &oout, &max_bins);
    char* sc = (char*)d_scratch;
    const int nb = std::min(nbins, max_bins);
    HIPCHK(launch_spectrum_bins(a, nx, ny, nb, (double*)(sc + obins), (double*)(sc + opart),
                                spectrum_partials(nx, ny), (double*)(sc + oout), E.stream));
    for (int i = nb; i < nbins; ++i) h_Ek[i] = 0.0;
    HIPCHK(hipMemcpyAsync(h_Ek, sc + obins, sizeof(double) * nb, hipMemcpyDeviceToHost, E.stream));
    double zz = 0;
    HIPCHK(hipMemcpyAsync(&zz, sc + oout, sizeof(double), hipMemcpyDeviceToHost, E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
    if (h_enstrophy) *h_enstrophy = 0.5 * zz;
    return RLBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free spectrum: the scratch of rlbm_spectrum in a file-scope
// device array.  Each device that runs it holds its own copy of the array
// (until the process ends); host code reaches a device's copy only through the
// address hipGetSymbolAddress returns for that device, taken once per device
// with the device current.  Every location the spectrum reads is written
// earlier in the same call, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)33 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array.
static int static_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RLBM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RLBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RLBM_OK;
}

int rlbm_spectrum_static(rlbm_ctx* ctx, double* h_Ek, int32_t nbins, double* h_enstrophy) {
    if (int rc = check_ctx(ctx)) return rc;
    Engine& E = ctx->e;
    if (!h_Ek || nbins < 1) return fail(RLBM_EINVAL, "bad spectrum arguments");
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != E.dev) return fail(RLBM_EINVAL, "call with the context's device current");
    size_t a, b, c, d, e, f;
    int mb = 0;
    const size_t need = spectrum_layout(E.lats[0].nx, E.lats[0].ny, &a, &b, &c, &d, &e, &f, &mb);
    if (need > kStaticScratchBytes)
        return fail(RLBM_ENOSPACE, "lattice too large for the static spectrum scratch "
                                   "(33 MiB: at most 2^20 sites)");
    void* p = nullptr;
    if (int rc = static_scratch(cur, &p)) return rc;
    return rlbm_spectrum(ctx, p, kStaticScratchBytes, h_Ek, nbins, h_enstrophy);
}

int rlbm_filtered_velocity(rlbm_ctx* ctx, void* d_scratch, size_t scratch_bytes, double k_lo,
                           double k_hi, double* d_ux, double* d_uy, double* h_mean_speed) {
    if (int rc = check_ctx(ctx)) return rc;
    Engine& E = ctx->e;
    if (!(k_lo >= 0.0) || !(k_hi >= k_lo)) return fail(RLBM_EINVAL, "band must satisfy 0 <= k_lo <= k_hi");
    const int nx = E.lats[0].nx, ny = E.lats[0].ny;
    double2* a = nullptr;
    int max_bins = 0;
    if (int rc = spectrum_transform(E, d_scratch, scratch_bytes, &a, &max_bins)) return rc;
    size_t oz2, otx, oty, obins, opart, oout;
    spectrum_layout(nx, ny, &oz2, &otx, &oty, &obins, &opart, &oout, &max_bins);
    char* sc = (char*)d_scratch;
    const double hi2 = std::isfinite(k_hi) ? k_hi * k_hi : HUGE_VAL;
    HIPCHK(launch_band_conj(a, nx, ny, k_lo * k_lo, hi2, E.stream));
    double2* other = a == (double2*)sc ? (double2*)(sc + oz2) : (double2*)sc;
    double2* w = fft2_forward(E, sc, a, other, otx, oty);
    if (!w) return fail(RLBM_EHIP, "FFT pass launch failed");
    HIPCHK(launch_unpack_speed(w, nx, ny, d_ux, d_uy, (double*)(sc + opart),
                               spectrum_partials(nx, ny), (double*)(sc + oout), E.stream));
    if (h_mean_speed) {
        double s = 0;
        HIPCHK(hipMemcpyAsync(&s, sc + oout, sizeof(double), hipMemcpyDeviceToHost, E.stream));
        HIPCHK(hipStreamSynchronize(E.stream));
        *h_mean_speed = s / ((double)nx * (double)ny);
    }
    return RLBM_OK;
}

int rlbm_state_bytes(const rlbm_ctx* ctx, size_t* h_bytes) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!h_bytes) return fail(RLBM_EINVAL, "NULL output");
    const Engine& E = ctx->e;
    *h_bytes = sizeof(SaveHeader) +
               (size_t)E.Q * E.hdesc[0].pitch * E.lats[0].ny * storage_bytes(E.storage);
    return RLBM_OK;
}

int rlbm_save(rlbm_ctx* ctx, void* h_buf, size_t bytes) {
    size_t need = 0;
    if (int rc = rlbm_state_bytes(ctx, &need)) return rc;
    if (!h_buf) return fail(RLBM_EINVAL, "NULL buffer");
    if (bytes < need) return fail(RLBM_ENOSPACE, "checkpoint buffer too small");
    Engine& E = ctx->e;
    SaveHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "RLBMSAV1", 8);
    h.version = 2;
    h.tau_mode = E.hdesc[0].tau_mode;
    h.stencil = E.stencil;
    h.storage = E.storage;
    h.nx = E.lats[0].nx;
    h.ny = E.lats[0].ny;
    h.Q = E.Q;
    h.step = E.step;
    h.tau = E.taus[0];
    h.cfl = E.lats[0].cfl;
    h.amplitude = E.frc[0].amplitude;
    h.k_lo = E.frc[0].k_lo;
    h.k_hi = E.frc[0].k_hi;
    h.seed = E.frc[0].seed;
    std::memcpy(h_buf, &h, sizeof(h));
    // the population buffer as stored (row bricks, padded columns included)
    const RealDesc& d = E.hdesc[0];
    char* dst = (char*)h_buf + sizeof(h);
    HIPCHK(hipMemcpyAsync(dst, d.buf[E.parity()], need - sizeof(h), hipMemcpyDeviceToHost,
                          E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
    return RLBM_OK;
}

int rlbm_load(rlbm_ctx* ctx, const void* h_buf, size_t bytes) {
    size_t need = 0;
    if (int rc = rlbm_state_bytes(ctx, &need)) return rc;
    if (!h_buf || bytes < need) return fail(RLBM_EINVAL, "checkpoint buffer missing or short");
    Engine& E = ctx->e;
    SaveHeader h;
    std::memcpy(&h, h_buf, sizeof(h));
    if (std::memcmp(h.magic, "RLBMSAV1", 8) != 0 || h.version != 2)
        return fail(RLBM_EINVAL, "not a checkpoint of this library");
    if (h.stencil != E.stencil || h.storage != E.storage || h.nx != E.lats[0].nx ||
        h.ny != E.lats[0].ny || h.Q != E.Q || h.tau != E.taus[0] || h.cfl != E.lats[0].cfl ||
        h.amplitude != E.frc[0].amplitude || h.k_lo != E.frc[0].k_lo ||
        h.k_hi != E.frc[0].k_hi || h.seed != E.frc[0].seed ||
        h.tau_mode != E.hdesc[0].tau_mode || h.step < 0)
        return fail(RLBM_EINVAL, "checkpoint of another configuration");
    E.step = h.step;
    HIPCHK(launch_reset(E.d_step, h.step, E.flips, E.d_flag, E.stream));
    const RealDesc& d = E.hdesc[0];
    const char* src = (const char*)h_buf + sizeof(h);
    HIPCHK(hipMemcpyAsync(d.buf[E.parity()], src, need - sizeof(h), hipMemcpyHostToDevice,
                          E.stream));
    if (int rc = E.prime_force_table()) return rc;
    HIPCHK(hipStreamSynchronize(E.stream));
    return RLBM_OK;
}

int engine_set_kernel(Engine& E, int32_t kind, int32_t param) {
    if (kind == RLBM_KERNEL_TILE) {
        if (param != 1 && param != 2 && param != 4 && param != 8)
            return fail(RLBM_EINVAL, "tile height must be 1, 2, 4 or 8");
        E.cfg[0].kind = kKernelTile;
        E.cfg[0].th = param;
        E.pairs = false;
    } else if (kind == RLBM_KERNEL_STAGED) {
        if (param != 0 && param != 4) return fail(RLBM_EINVAL, "staged tile height must be 4 (or 0)");
        if (E.smode == kStreamHalo2)
            return fail(RLBM_EUNSUPPORTED, "the staged form needs cfl <= 1");
        E.cfg[0].kind = kKernelStaged;
        E.cfg[0].th = 4;
        E.pairs = false;
    } else if (kind == RLBM_KERNEL_MARCH_PAIRS) {
        if (param < 0 || param > 65536) return fail(RLBM_EINVAL, "segment length must be in [0, 65536]");
        if (E.smode == kStreamHalo2)
            return fail(RLBM_EUNSUPPORTED, "the row-marching forms need cfl <= 1");
        if (!E.kind_fits(kKernelMarchPair))
            return fail(RLBM_EUNSUPPORTED, "the row-marching forms need forcing modes with |kx| <= 63");
        if (E.storage != RLBM_F16S && E.storage != RLBM_BF16S)
            return fail(RLBM_EUNSUPPORTED, "the paired marching form is for 16-bit storage");
        if (!E.even_nx())
            return fail(RLBM_EUNSUPPORTED, "the paired marching form needs an even nx");
        E.cfg[0].kind = kKernelMarchPair;
        E.cfg[0].seglen_req = param;
        E.pairs = false;
    } else if (kind == RLBM_KERNEL_MARCH || kind == RLBM_KERNEL_MARCH2) {
        if (param < 0 || param > 65536) return fail(RLBM_EINVAL, "segment length must be in [0, 65536]");
        if (E.smode == kStreamHalo2)
            return fail(RLBM_EUNSUPPORTED, "the row-marching forms need cfl <= 1");
        if (!E.kind_fits(kKernelMarch))
            return fail(RLBM_EUNSUPPORTED, "the row-marching forms need forcing modes with |kx| <= 63");
        if (kind == RLBM_KERNEL_MARCH) {
            E.cfg[0].kind = kKernelMarch;
            E.cfg[0].seglen_req = param;
            E.pairs = false;
        } else {
            // the two-step form reads input rows up to two past a segment's
            // last row and wraps them by one period: every lattice needs ny >= 3
            for (const rlbm_lattice& l : E.lats)
                if (l.ny < 3) return fail(RLBM_EUNSUPPORTED, "the two-step form needs ny >= 3");
            E.cfg[1].kind = kKernelMarch2;
            E.cfg[1].seglen_req = param;
            E.pairs = true;
        }
    } else {
        return fail(RLBM_EINVAL, "unknown kernel kind");
    }
    E.kind_auto = false;
    return E.configure_tiles();
}

int rlbm_set_kernel(rlbm_ctx* ctx, int32_t kind, int32_t param) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_set_kernel(ctx->e, kind, param);
}

int rlbm_set_tile(rlbm_ctx* ctx, int32_t th) { return rlbm_set_kernel(ctx, RLBM_KERNEL_TILE, th); }

int engine_get_kernel(const Engine& E, int32_t* h_kind, int32_t* h_param) {
    if (!h_kind || !h_param) return fail(RLBM_EINVAL, "NULL output");
    if (E.pairs) {
        *h_kind = RLBM_KERNEL_MARCH2;
        *h_param = E.cfg[1].seglen;
    } else if (E.cfg[0].kind == kKernelMarch) {
        *h_kind = RLBM_KERNEL_MARCH;
        *h_param = E.cfg[0].seglen;
    } else if (E.cfg[0].kind == kKernelStaged) {
        *h_kind = RLBM_KERNEL_STAGED;
        *h_param = E.cfg[0].th;
    } else if (E.cfg[0].kind == kKernelMarchPair) {
        *h_kind = RLBM_KERNEL_MARCH_PAIRS;
        *h_param = E.cfg[0].seglen;
    } else {
        *h_kind = RLBM_KERNEL_TILE;
        *h_param = E.cfg[0].th;
    }
    return RLBM_OK;
}

// Time every candidate form for `steps` steps (advancing the state, which no
// form changes: results are bitwise the same) and keep the fastest.
int engine_autotune(Engine& E, int32_t steps, int32_t* h_th) {
    if (steps < 1) return fail(RLBM_EINVAL, "steps must be >= 1");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    steps += steps & 1;                           // whole pairs for the two-step form
    float best = 1e30f;
    int best_kind = -1, best_param = 0;
    // (kind, parameter): tile heights; marching forms with the automatic
    // segment length (0: about one segment per resident wavefront) and with
    // segments 2x (-1), 3/2 x (-2), 1/2 x (-3) and 3/4 x (-4) as long; which
    // of these runs fastest depends on how the rounds of segments fill the
    // chip (measured: 16-bit storage at 2048^2, 105 us at 8 rows, 127 us at 11);
    // the two-step form with segments of 12 (its default), 8, 10, 16, 18, 20,
    // 24 and 32 rows (FP32 2048^2: 149 us at 18 rows, 152 at 12, 170 at 15)
    const int cand[23][2] = {{RLBM_KERNEL_TILE, 1},   {RLBM_KERNEL_TILE, 2},
                             {RLBM_KERNEL_TILE, 4},   {RLBM_KERNEL_TILE, 8},
                             {RLBM_KERNEL_STAGED, 4},
                             {RLBM_KERNEL_MARCH, 0},  {RLBM_KERNEL_MARCH, -1},
                             {RLBM_KERNEL_MARCH, -2}, {RLBM_KERNEL_MARCH, -3},
                             {RLBM_KERNEL_MARCH, -4},
                             {RLBM_KERNEL_MARCH_PAIRS, 0},  {RLBM_KERNEL_MARCH_PAIRS, -1},
                             {RLBM_KERNEL_MARCH_PAIRS, -2}, {RLBM_KERNEL_MARCH_PAIRS, -3},
                             {RLBM_KERNEL_MARCH_PAIRS, -4},
                             {RLBM_KERNEL_MARCH2, 0},  {RLBM_KERNEL_MARCH2, 8},
                             {RLBM_KERNEL_MARCH2, 10}, {RLBM_KERNEL_MARCH2, 16},
                             {RLBM_KERNEL_MARCH2, 18}, {RLBM_KERNEL_MARCH2, 20},
                             {RLBM_KERNEL_MARCH2, 24}, {RLBM_KERNEL_MARCH2, 32}};
    int auto_seg[5] = {0, 0, 0, 0, 0};
    int tried[23][2];
    int n_tried = 0;
    const bool bits16 = E.storage == RLBM_F16S || E.storage == RLBM_BF16S;
    int min_ny = 65536;
    for (const rlbm_lattice& l : E.lats) min_ny = std::min(min_ny, (int)l.ny);
    int rc = RLBM_OK;
    for (const auto& c : cand) {
        if (c[0] != RLBM_KERNEL_TILE && E.smode == kStreamHalo2) continue;
        if (c[0] == RLBM_KERNEL_MARCH_PAIRS && (!bits16 || !E.even_nx())) continue;
        if (c[0] != RLBM_KERNEL_TILE && c[0] != RLBM_KERNEL_STAGED && !E.kind_fits(kKernelMarch))
            continue;
        if (c[0] == RLBM_KERNEL_MARCH2 && min_ny < 3) continue;
        const int a = auto_seg[c[0]];
        int param = c[1];
        if (c[1] < 0) {
            const int scaled[4] = {2 * a, (3 * a + 1) / 2, (a + 1) / 2, (3 * a + 3) / 4};
            param = std::max(2, scaled[-c[1] - 1]);
        }
        bool seen = false;                         // a short lattice maps several to one
        for (int i = 0; i < n_tried; ++i) seen |= tried[i][0] == c[0] && tried[i][1] == param;
        if (seen) continue;
        if ((rc = engine_set_kernel(E, c[0], param))) break;
        int32_t k = 0, p = 0;
        engine_get_kernel(E, &k, &p);
        if (c[1] == 0) auto_seg[c[0]] = p;
        tried[n_tried][0] = c[0];
        tried[n_tried][1] = c[1] == 0 ? p : param;
        ++n_tried;
        if ((rc = E.run(2))) break;
        if (hipEventRecord(e0, E.stream) != hipSuccess) { rc = fail(RLBM_EHIP, "event record failed"); break; }
        if ((rc = E.run(steps))) break;
        float ms = 0;
        if (hipEventRecord(e1, E.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(RLBM_EHIP, "event timing failed");
            break;
        }
        if (ms < best) {
            best = ms;
            best_kind = k;
            best_param = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (h_th) *h_th = best_kind == RLBM_KERNEL_TILE || best_kind == RLBM_KERNEL_STAGED ? best_param
                                                                                     : -best_param;
    static_assert(RLBM_KERNEL_MARCH_PAIRS < 5, "auto_seg is indexed by the kernel kind");
    return engine_set_kernel(E, best_kind, best_param);
}

int rlbm_autotune(rlbm_ctx* ctx, int32_t steps, int32_t* h_th) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_autotune(ctx->e, steps, h_th);
}

int rlbm_get_kernel(const rlbm_ctx* ctx, int32_t* h_kind, int32_t* h_param) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_get_kernel(ctx->e, h_kind, h_param);
}

int rlbm_set_graph_chunk(rlbm_ctx* ctx, int32_t chunk) {
    if (int rc = check_ctx(ctx)) return rc;
    if (chunk < 0 || chunk > 4096) return fail(RLBM_EINVAL, "chunk must be in [0, 4096]");
    ctx->e.graph_chunk = chunk;
    return RLBM_OK;
}

int rlbm_set_relaxation(rlbm_ctx* ctx, int32_t mode) {
    if (int rc = check_ctx(ctx)) return rc;
    return engine_set_relaxation(ctx->e, mode);
}

int rlbm_profile_step_kernel(rlbm_ctx* ctx, int64_t n, double* h_ms) {
    if (int rc = check_ctx(ctx)) return rc;
    if (!h_ms) return fail(RLBM_EINVAL, "NULL output");
    return ctx->e.profile(n, h_ms);
}

void rlbm_destroy(rlbm_ctx* ctx) { delete ctx; }

// ---- ensemble -----------------------------------------------------------------
int rlbm_batch_workspace_bytes(int32_t n_real, const rlbm_lattice* lats, int stencil, int storage,
                               const rlbm_forcing* forcings, size_t* h_bytes) {
    return engine_bytes(n_real, lats, stencil, storage, forcings, h_bytes);
}

int rlbm_batch_init(rlbm_batch** out, int32_t n_real, const rlbm_lattice* lats,
                    const double* taus, int stencil, const rlbm_forcing* forcings, int storage,
                    void* d_workspace, size_t ws_bytes, void* hip_stream) {
    if (!out) return fail(RLBM_EINVAL, "out is NULL");
    *out = nullptr;
    rlbm_batch* b = new (std::nothrow) rlbm_batch();
    if (!b) return fail(RLBM_EINVAL, "out of host memory");
    int rc = engine_init(b->e, n_real, lats, taus, stencil, forcings, storage, d_workspace,
                         ws_bytes, hip_stream);
    if (rc) { delete b; return rc; }
    *out = b;
    return RLBM_OK;
}

int rlbm_batch_set_state(rlbm_batch* b, int32_t r, const double* d_e, const double* d_ux,
                         const double* d_uy) {
    if (int rc = check_ctx(b)) return rc;
    if (r < 0 || r >= b->e.n_real) return fail(RLBM_EINVAL, "realization out of range");
    if (b->e.step != 0) return fail(RLBM_EINVAL, "set the ensemble state before the first step");
    return engine_set_state(b->e, r, d_e, d_ux, d_uy, false);
}

int rlbm_batch_step(rlbm_batch* b, int64_t n) {
    if (int rc = check_ctx(b)) return rc;
    return b->e.run(n);
}

int rlbm_batch_check(rlbm_batch* b) {
    if (int rc = check_ctx(b)) return rc;
    return engine_check(b->e);
}

int rlbm_batch_fields(rlbm_batch* b, int32_t r, double* d_e, double* d_ux, double* d_uy,
                      double* d_T) {
    if (int rc = check_ctx(b)) return rc;
    if (r < 0 || r >= b->e.n_real) return fail(RLBM_EINVAL, "realization out of range");
    return engine_fields(b->e, r, d_e, d_ux, d_uy, d_T, nullptr);
}

int rlbm_batch_get_populations(rlbm_batch* b, int32_t r, double* d_out) {
    if (int rc = check_ctx(b)) return rc;
    if (r < 0 || r >= b->e.n_real || !d_out) return fail(RLBM_EINVAL, "bad arguments");
    Engine& E = b->e;
    HIPCHK(launch_get_populations(E.d_desc, r, E.storage, E.stencil, E.lats[r].nx, E.lats[r].ny, d_out,
                                  E.parity(), E.stream));
    return RLBM_OK;
}

int rlbm_batch_set_graph_chunk(rlbm_batch* b, int32_t chunk) {
    if (int rc = check_ctx(b)) return rc;
    if (chunk < 0 || chunk > 4096) return fail(RLBM_EINVAL, "chunk must be in [0, 4096]");
    b->e.graph_chunk = chunk;
    return RLBM_OK;
}

int rlbm_batch_set_kernel(rlbm_batch* b, int32_t kind, int32_t param) {
    if (int rc = check_ctx(b)) return rc;
    return engine_set_kernel(b->e, kind, param);
}

int rlbm_batch_step_count(const rlbm_batch* b, int64_t* h_steps) {
    if (int rc = check_ctx(b)) return rc;
    if (!h_steps) return fail(RLBM_EINVAL, "NULL output");
    *h_steps = b->e.step;
    return RLBM_OK;
}

int rlbm_batch_get_kernel(const rlbm_batch* b, int32_t* h_kind, int32_t* h_param) {
    if (int rc = check_ctx(b)) return rc;
    return engine_get_kernel(b->e, h_kind, h_param);
}

int rlbm_batch_autotune(rlbm_batch* b, int32_t steps, int32_t* h_th) {
    if (int rc = check_ctx(b)) return rc;
    return engine_autotune(b->e, steps, h_th);
}

int rlbm_batch_set_relaxation(rlbm_batch* b, int32_t mode) {
    if (int rc = check_ctx(b)) return rc;
    return engine_set_relaxation(b->e, mode);
}

void rlbm_batch_destroy(rlbm_batch* b) { delete b; }

}  // extern "C"
