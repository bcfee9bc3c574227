// dpml.hip -- host side of the discrete-PML wave stepper for MI355X (gfx950):
// argument validation, workspace carve-up, damping tables, kernel launches
// and the C ABI declared in include/dpml.h.
//
// The scheme is Eq. (DiscretePML a-c) of Chern, "A Reflectionless Discrete
// Perfectly Matched Layer", stepped with leapfrog for U and a forward step
// for the auxiliaries, all right-hand sides at time level n (see
// dpml_kernels.hpp for the per-cell arithmetic).
#include "dpml.h"
#include "dpml_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <mutex>
#include <vector>

#include "dpml_host.hpp"

using namespace dpmlh;

namespace {










template <typename T>
int launch_step(dpml *H, T *hist = nullptr, T *uout = nullptr)
{
    const Layout &L = H->L;
    dpmlk::StepArgs<T> p = make_args<T>(H);
    p.hist = hist;
    p.uout = uout;
    const unsigned B = (unsigned)L.batch;
    const bool multi = pass_depth(H->variant, H->tile_rows) >= 2;
    int variant = (H->variant == DPML_VARIANT_AUTO || multi) ? DPML_VARIANT_CELL : H->variant;
    // 3D single steps of the multi-step variants march like MARCH
    if (L.ndim == 3 && multi) variant = DPML_VARIANT_MARCH;
    if (L.ndim == 3 && variant != DPML_VARIANT_CELL)
        return launch_march3d<T>(H, p, variant == DPML_VARIANT_MARCH ? 4 : 2);
    const int slot = timed_begin(H, DPML_KERNEL_STEP, step_bytes(H, (double)L.ncell, aux_cells(L)));
    if (variant == DPML_VARIANT_CELL) {
        // tile_rows selects the block shape: TH rows of 256/TH cells (TH = 1, 2, 4, 8)
        const int th = (H->tile_rows == 1 || H->tile_rows == 2 || H->tile_rows == 8) ? H->tile_rows : 4;
        const int tw = 256 / th;
        p.tiles_x = (int)((L.N[0] + tw - 1) / tw);
        p.tiles_y = (int)((L.N[1] + th - 1) / th);
        p.n_tiles = p.tiles_x * p.tiles_y * (int)(L.ndim == 3 ? L.N[2] : 1);
        dim3 grid((unsigned)round8(p.n_tiles), B), block(256);
#define DPML_CELL_LAUNCH(TH_)                                                                    \
        if (L.ndim == 2) hipLaunchKernelGGL((dpmlk::k_step_cell<T, 2, TH_>), grid, block, 0, H->stream, p); \
        else hipLaunchKernelGGL((dpmlk::k_step_cell<T, 3, TH_>), grid, block, 0, H->stream, p);
        if (th == 1) { DPML_CELL_LAUNCH(1) }
        else if (th == 2) { DPML_CELL_LAUNCH(2) }
        else if (th == 8) { DPML_CELL_LAUNCH(8) }
        else { DPML_CELL_LAUNCH(4) }
#undef DPML_CELL_LAUNCH
    } else {
        // vector width: 8 bytes per thread when the rows allow it
        constexpr int VX = sizeof(T) == 4 ? 2 : 1;
        const int vx = (L.N[0] % VX == 0) ? VX : 1;
        const bool grouped = variant == DPML_VARIANT_MARCH;
        p.tile_rows = H->tile_rows > 0 ? H->tile_rows : 16;
        p.tiles_x = (int)((L.N[0] + 256 * vx - 1) / (256 * vx));
        const int tiles_y = (int)((L.N[1] + p.tile_rows - 1) / p.tile_rows);
        p.n_tiles = p.tiles_x * tiles_y;
        dim3 grid((unsigned)round8(p.n_tiles), B), block(256);
        if (vx == 2 && grouped)
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, (sizeof(T) == 4 ? 2 : 1), 4>), grid, block, 0, H->stream, p);
        else if (vx == 2)
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, (sizeof(T) == 4 ? 2 : 1), 1>), grid, block, 0, H->stream, p);
        else if (grouped)
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, 1, 4>), grid, block, 0, H->stream, p);
        else
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, 1, 1>), grid, block, 0, H->stream, p);
    }
    timed_end(H, slot);
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}




// Columns per lane of the multi-step core kernels.
int multistep_vx(const Layout &L) { return L.dtype == DPML_F32 ? 4 : 2; }

// Core rectangle of a multi-step pass over `levels` levels: cells whose
// (levels-1)-cell halo is free of damping terms, inside [lo+levels,
// lo+n+1-levels) per axis (the undamped cells are [lo+1, lo+n)); along x it
// starts on a multiple of the kernel's vector width and spans a multiple of
// it.  An axis without a layer is core over its whole (periodic) extent.
void core_rect(const Layout &L, int levels, int r[4])
{
    const int vx = multistep_vx(L);
    for (int a = 0; a < 2; ++a) {
        if (L.M[a] == 0) {
            r[2 * a] = 0;
            r[2 * a + 1] = (int)L.N[a];
            continue;
        }
        int b0 = L.lo[a] + levels, b1 = (int)(L.lo[a] + L.n[a] + 1 - levels);
        if (a == 0) {
            b0 = (b0 + vx - 1) / vx * vx;
            b1 = b1 > b0 ? b0 + (b1 - b0) / vx * vx : b0;
        }
        r[2 * a] = b0;
        r[2 * a + 1] = std::max(b0, b1);
    }
}




// Levels per pass this handle may take right now: the variant's depth, fewer
// for the last steps of a run or where the core of that depth is empty, or 1.
bool frame_fused(const dpml *H);

int multistep_levels(const dpml *H, int64_t nsteps)
{
    const Layout &L = H->L;
    if (L.ndim == 3) return multistep_levels3d(H, nsteps);
    if (!walls_allow_multistep(L)) return 1;
    if (H->recording && H->plane_axis >= 0) return 1;
    // sources and receivers: passes of 4 .. 8 levels (the deep cores form
    // them; the frame's per-step launches record), at most 32 sources, each
    // at least levels-1 cells inside the core (the frame's steps then add
    // none), receivers on distinct cells
    const bool taps = H->ns > 0 || (H->recording && H->nr > 0);
    if (taps && (H->ns > 32 || frame_fused(H) || (H->recording && H->rec_dups))) return 1;
    int want = pass_depth(H->variant, H->tile_rows);
    if (want > nsteps) want = (int)nsteps;
    // the core kernels wrap halo rows once: each extent must hold its halos
    if (L.N[0] < 8 || L.N[1] < 8) return 1;
    for (; want >= 2; --want) {
        int r[4];
        core_rect(L, want, r);
        if (r[1] - r[0] < 1 || r[3] - r[2] < 1) continue;
        if (!taps) return want;
        if (want < 4) return 1;
        bool inside = true;
        for (int64_t cell : H->src_sorted) {
            const int64_t c = cell % L.ncell;
            const int x = (int)(c % L.N[0]), y = (int)(c / L.N[0]);
            inside &= x >= r[0] + want - 1 && x < r[1] - (want - 1) && y >= r[2] + want - 1 && y < r[3] - (want - 1);
        }
        if (inside) return want;
    }
    return 1;
}

// Rows per span of the marching frame steps of a problem set, and rows
// whose loads a wave issues together (measured on the 256-problem set).
constexpr int kFrameRows = 16;
constexpr int kFrameGroup = 8;

// The spans (64 columns x up to `rows` rows, counted across the
// periodic wrap) covering everything outside the rectangle S = [S0, S1) x
// [S2, S3) of a 2D grid: the rows outside S on every column, and S's rows on
// the columns outside S (one strip across the wrap).  An axis where S spans
// the whole grid adds nothing.
void frame_spans(const Layout &L, const int S[4], int prob, std::vector<dpmlk::Span2> &out, int rows = kFrameRows)
{
    const int NX = (int)L.N[0], NY = (int)L.N[1];
    auto rect = [&](int xs, int xe, int ys, int ye) {
        for (int y = ys; y < ye; y += rows)
            for (int x = xs; x < xe; x += 64)
                out.push_back({prob, x, std::min(x + 64, xe), y, std::min(y + rows, ye), 0, 0, 0});
    };
    if (S[3] - S[2] < NY) rect(0, NX, S[3], S[2] + NY);
    if (S[1] - S[0] < NX) rect(S[1], S[0] + NX, S[2], S[3]);
}

// Frame form of the multi-step variants, bits 16-19 of tile_rows: 0 the
// frame's steps one thread per cell; 1 .. 14 wave marches over spans of that
// many rows (periodic grids only: with walls the frame is one thread per
// cell); kFrameFused all of a pass's frame steps in one launch.
constexpr int kFrameFused = 15;

bool frame_fused(const dpml *H) { return ((H->tile_rows >> 16) & 0xF) == kFrameFused; }

int frame_span_rows(const dpml *H)
{
    const int f = (H->tile_rows >> 16) & 0xF;
    return (H->L.wall[0] || H->L.wall[1] || f == kFrameFused) ? 0 : f;
}

// Tile shape of the fused frame kernel per element type.
template <typename T>
struct FusedTile {
    static constexpr int TX = 64, TY = 8;
};

// The fused frame's tiles for passes of `levels` levels: the TX x TY tiles of
// a fixed grid that meet everything outside the core shrunk by one.
int ensure_fused(dpml *H, int levels, int TX, int TY)
{
    const int q = levels - 2;
    if (H->n_ffused[q] >= 0) return DPML_OK;
    const Layout &L = H->L;
    int r[4];
    core_rect(L, levels, r);
    const int in[4] = {r[0] + 1, r[1] - 1, r[2] + 1, r[3] - 1};
    const int tx = (int)((L.N[0] + TX - 1) / TX), ty = (int)((L.N[1] + TY - 1) / TY);
    std::vector<dpmlk::TileRef> t;
    for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x) {
            const int xa = x * TX, xb = std::min<int>(xa + TX, (int)L.N[0]);
            const int ya = y * TY, yb = std::min<int>(ya + TY, (int)L.N[1]);
            const bool inside = xa >= in[0] && xb <= in[1] && ya >= in[2] && yb <= in[3];
            if (!inside) t.push_back({0, x, y, 0});
        }
    H->n_ffused[q] = (int64_t)t.size();
    if (t.empty()) return DPML_OK;
    HIP_TRY(H, hipMalloc((void **)&H->d_ffused[q], t.size() * sizeof(dpmlk::TileRef)));
    HIP_TRY(H, hipMemcpy(H->d_ffused[q], t.data(), t.size() * sizeof(dpmlk::TileRef), hipMemcpyHostToDevice));
    return DPML_OK;
}

int ensure_frame(dpml *H, int levels, int shrink)
{
    const int q = levels - 2;
    const Layout &L = H->L;
    int r[4];
    core_rect(L, levels, r);
    r[0] += shrink;
    r[1] -= shrink;
    r[2] += shrink;
    r[3] -= shrink;
    const int fr = frame_span_rows(H);
    if (fr > 0) {
        if (H->fspan_rows != fr) {                    // span lists of another height
            for (int a = 0; a < kMaxLevels - 1; ++a)
                for (int b = 0; b < kMaxLevels; ++b) {
                    if (H->d_fspan[a][b]) HIP_TRY(H, hipFree(H->d_fspan[a][b]));
                    H->d_fspan[a][b] = nullptr;
                    H->n_fspan[a][b] = -1;
                }
            H->fspan_rows = fr;
        }
        if (H->n_fspan[q][shrink] >= 0) return DPML_OK;
        std::vector<dpmlk::Span2> sp;
        frame_spans(L, r, 0, sp, fr);
        H->n_fspan[q][shrink] = (int64_t)sp.size();
        if (sp.empty()) return DPML_OK;
        HIP_TRY(H, hipMalloc((void **)&H->d_fspan[q][shrink], sp.size() * sizeof(dpmlk::Span2)));
        HIP_TRY(H, hipMemcpy(H->d_fspan[q][shrink], sp.data(), sp.size() * sizeof(dpmlk::Span2), hipMemcpyHostToDevice));
        return DPML_OK;
    }
    if (H->n_frame[q][shrink] >= 0) return DPML_OK;
    // one thread per cell over 64 x 4 tiles
    const int tx = (int)((L.N[0] + 63) / 64), ty = (int)((L.N[1] + 3) / 4);
    std::vector<dpmlk::TileRef> t;
    for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x) {
            const int xa = x * 64, xb = std::min<int>(xa + 64, (int)L.N[0]);
            const int ya = y * 4, yb = std::min<int>(ya + 4, (int)L.N[1]);
            const bool inside = xa >= r[0] && xb <= r[1] && ya >= r[2] && yb <= r[3];
            if (!inside) t.push_back({0, x, y, 0});
        }
    H->n_frame[q][shrink] = (int64_t)t.size();
    if (t.empty()) return DPML_OK;
    HIP_TRY(H, hipMalloc((void **)&H->d_frame[q][shrink], t.size() * sizeof(dpmlk::TileRef)));
    HIP_TRY(H, hipMemcpy(H->d_frame[q][shrink], t.data(), t.size() * sizeof(dpmlk::TileRef), hipMemcpyHostToDevice));
    return DPML_OK;
}

// Everything a multi-step pass over `levels` levels needs before it can be
// enqueued (or captured): the frame tables and the side stream with its
// fork/join events.
int ensure_multistep(dpml *H, int levels)
{
    if (H->L.ndim == 3) return ensure_side(H);
    if (frame_fused(H)) {
        const bool f32 = H->L.dtype == DPML_F32;
        int rc = ensure_fused(H, levels, f32 ? FusedTile<float>::TX : FusedTile<double>::TX,
                              f32 ? FusedTile<float>::TY : FusedTile<double>::TY);
        return rc ? rc : ensure_side(H);
    }
    for (int sh = 0; sh < levels; ++sh) {
        int rc = ensure_frame(H, levels, sh);
        if (rc) return rc;
    }
    return ensure_side(H);
}

// Receiver tables of the 2D passes with receivers: per (member, row) a
// column map of receiver indices in a pool (built once per registration),
// and for passes of `levels` levels over the core r the receivers sorted by
// how deep they lie in the core (min distance to its edges; negative
// outside), with the frame's share at level l = those less than levels-l
// deep (the core records the rest).
// Per (member, row) index into a pool of per-row column maps of the
// registered receivers (receiver index or -1).
int ensure_rmap(dpml *H)
{
    const Layout &L = H->L;
    const int NX = (int)L.N[0], NY = (int)L.N[1];
    if (!H->d_rmap) {
        std::vector<int32_t> rmap((size_t)(L.batch * NY), -1), pool;
        for (int64_t i = 0; i < (int64_t)H->rec_host.size(); ++i) {
            const int64_t cell = H->rec_host[i], b = cell / L.ncell, c = cell % L.ncell;
            const int64_t key = b * NY + c / NX;
            if (rmap[(size_t)key] < 0) {
                rmap[(size_t)key] = (int32_t)pool.size();
                pool.resize(pool.size() + (size_t)NX, -1);
            }
            pool[(size_t)rmap[(size_t)key] + (size_t)(c % NX)] = (int32_t)i;
        }
        HIP_TRY(H, hipMalloc((void **)&H->d_rmap, rmap.size() * sizeof(int32_t)));
        HIP_TRY(H, hipMalloc((void **)&H->d_rpool, std::max<size_t>(pool.size(), 1) * sizeof(int32_t)));
        HIP_TRY(H, hipMemcpy(H->d_rmap, rmap.data(), rmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        if (!pool.empty())
            HIP_TRY(H, hipMemcpy(H->d_rpool, pool.data(), pool.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    return DPML_OK;
}

int ensure_taps(dpml *H, int levels, const int r[4])
{
    const Layout &L = H->L;
    const int NX = (int)L.N[0];
    int rc = ensure_rmap(H);
    if (rc) return rc;
    const int q = levels - 2;
    if (!H->d_frec_cells[q]) {
        const int64_t nr = (int64_t)H->rec_host.size();
        std::vector<int64_t> order((size_t)nr);
        std::vector<int> depth((size_t)nr);
        for (int64_t i = 0; i < nr; ++i) {
            const int64_t c = H->rec_host[i] % L.ncell;
            const int x = (int)(c % NX), y = (int)(c / NX);
            depth[i] = std::min(std::min(x - r[0], r[1] - 1 - x), std::min(y - r[2], r[3] - 1 - y));
            order[i] = i;
        }
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return depth[a] < depth[b]; });
        std::vector<int64_t> cells((size_t)nr);
        std::vector<int32_t> idx((size_t)nr);
        for (int64_t k = 0; k < nr; ++k) {
            cells[k] = H->rec_host[order[k]];
            idx[k] = (int32_t)order[k];
        }
        for (int l = 1; l <= levels; ++l) {
            int64_t cnt = 0;
            while (cnt < nr && depth[order[cnt]] < levels - l) ++cnt;
            H->frec_count[q][l] = cnt;
        }
        HIP_TRY(H, hipMalloc((void **)&H->d_frec_cells[q], (size_t)std::max<int64_t>(nr, 1) * sizeof(int64_t)));
        HIP_TRY(H, hipMalloc((void **)&H->d_frec_idx[q], (size_t)std::max<int64_t>(nr, 1) * sizeof(int32_t)));
        HIP_TRY(H, hipMemcpy(H->d_frec_cells[q], cells.data(), (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice));
        HIP_TRY(H, hipMemcpy(H->d_frec_idx[q], idx.data(), (size_t)nr * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    return DPML_OK;
}

// Release the receiver tables (receivers re-registered, or destroy).
void free_taps(dpml *H)
{
    if (H->d_rmap) (void)hipFree(H->d_rmap);
    if (H->d_rpool) (void)hipFree(H->d_rpool);
    H->d_rmap = H->d_rpool = nullptr;
    if (H->d_adj_frec_cells) (void)hipFree(H->d_adj_frec_cells);
    if (H->d_adj_frec_order) (void)hipFree(H->d_adj_frec_order);
    H->d_adj_frec_cells = nullptr;
    H->d_adj_frec_order = nullptr;
    H->n_adj_frec = -1;
    for (int q = 0; q < kMaxLevels - 1; ++q) {
        if (H->d_frec_cells[q]) (void)hipFree(H->d_frec_cells[q]);
        if (H->d_frec_idx[q]) (void)hipFree(H->d_frec_idx[q]);
        H->d_frec_cells[q] = nullptr;
        H->d_frec_idx[q] = nullptr;
    }
}

// The fused frame kernel of a pass of 2 .. kMaxLevels levels.
template <typename T>
void launch_fused(int levels, dim3 grid, hipStream_t st, const dpmlk::StepArgs<T> &p, T *pen, T *fin,
                  const dpmlk::TileRef *tiles, int n)
{
    constexpr int TX = FusedTile<T>::TX, TY = FusedTile<T>::TY;
    const dim3 block(256);
#define DPML_FUSED(D_) \
    hipLaunchKernelGGL((dpmlk::k_frame_fused2d<T, D_, TX, TY>), grid, block, 0, st, p, pen, fin, tiles, n)
    switch (levels) {
    case 2: DPML_FUSED(2); break;
    case 3: DPML_FUSED(3); break;
    case 4: DPML_FUSED(4); break;
    case 5: DPML_FUSED(5); break;
    case 6: DPML_FUSED(6); break;
    case 7: DPML_FUSED(7); break;
    default: DPML_FUSED(8); break;
    }
#undef DPML_FUSED
}

// The core kernel of a pass of 4 .. kMaxLevels levels (pf: the next load
// group issued ahead).
template <typename T, int VX, int G, bool C2>
void launch_coreN(int levels, bool pf, dim3 grid, hipStream_t st, const dpmlk::StepArgs<T> &p, T *pen, T *fin,
                  const int r[4], int strips, int n_waves, const dpmlk::Taps2<T> &tp)
{
    const dim3 block(256);
#define DPML_CORE_N(NL)                                                                                        \
    if (pf)                                                                                                    \
        hipLaunchKernelGGL((dpmlk::k_stepN_march<T, VX, G, C2, NL, true>), grid, block, 0, st, p, pen, fin, r[0], \
                           r[1], r[2], r[3], strips, n_waves, tp);                                             \
    else                                                                                                       \
        hipLaunchKernelGGL((dpmlk::k_stepN_march<T, VX, G, C2, NL, false>), grid, block, 0, st, p, pen, fin, r[0], \
                           r[1], r[2], r[3], strips, n_waves, tp)
    switch (levels) {
    case 4: DPML_CORE_N(4); break;
    case 5: DPML_CORE_N(5); break;
    case 6: DPML_CORE_N(6); break;
    case 7: DPML_CORE_N(7); break;
    default: DPML_CORE_N(8); break;
    }
#undef DPML_CORE_N
}

// `levels` (2 .. kMaxLevels) steps.  The core kernel runs on the handle's stream;
// the frame takes `levels` ordinary steps on the side stream at the same
// time, step j (1-based) over everything outside the core shrunk by
// levels - j cells, which is where the later frame steps need level j.  The
// core writes no level-j value on those cells, so every cell of every
// buffer has one writer.  The pass ends with the handle's stream waiting
// for the side stream.  With `hist`, level l goes to hist + (l-1) * hstride
// (whole batch levels; every level kept: passes of 2 or 4 .. kMaxLevels
// levels, the frame's steps one launch per level) and the fields then point
// there.
template <typename T>
int launch_multistep(dpml *H, int levels, T *hist = nullptr, int64_t hstride = 0)
{
    const Layout &L = H->L;
    const unsigned B = (unsigned)L.batch;
    const int q = levels - 2;
    // buffers: A = U^n, Bv = U^{n-1}, then U^{n+1} .. U^{n+levels} in the spares
    T *A = (T *)H->u_now, *Bv = (T *)H->u_old;
    T *nxt[kMaxLevels] = {};
    int k = 0;
    if (hist) {
        if (levels == 3 || frame_fused(H)) return H->fail(DPML_EINVAL, "a history pass of this shape");
        for (; k < levels; ++k) nxt[k] = hist + (int64_t)k * hstride;
    }
    for (int i = 0; i < L.n_ubuf && k < levels; ++i) {
        void *b = H->at(L.off_u[i]);
        if (b != H->u_now && b != H->u_old) nxt[k++] = (T *)b;
    }
    if (k < levels) return H->fail(DPML_EINVAL, "not enough field buffers for a multi-step pass");
    int r[4];
    core_rect(L, levels, r);
    constexpr int VX = sizeof(T) == 4 ? 4 : 2;
    const int HL = (levels + VX - 1) / VX;                      // halo lanes per strip side
    // tile_rows: rows per wave in the low 12 bits (0: 8), loads issued G rows at a
    // time with G in the bits above (0: 2)
    const int rows = (H->tile_rows & 0xFFF) > 0 ? (H->tile_rows & 0xFFF) : 8;
    const int G = ((H->tile_rows >> 12) & 0xF) > 0 ? ((H->tile_rows >> 12) & 0xF) : 2;
    const int strips = (r[1] - r[0] + (64 - 2 * HL) * VX - 1) / ((64 - 2 * HL) * VX);
    const int n_waves = strips * ((r[3] - r[2] + rows - 1) / rows);
    const dim3 block(256);
    const double core = (double)(r[1] - r[0]) * (double)(r[3] - r[2]);
    // sources and receivers of this pass (passes of 4 .. 8 levels only)
    dpmlk::Taps2<T> tp{};
    const bool rec = H->recording && H->nr > 0;
    if (H->ns > 0 || rec) {
        if (levels < 4) return H->fail(DPML_EINVAL, "sources or receivers in a pass of fewer than 4 levels");
        if (rec) {
            int rc = ensure_taps(H, levels, r);
            if (rc) return rc;
            tp.nr = (int32_t)H->nr;
            tp.rmap = H->d_rmap;
            tp.rpool = H->d_rpool;
            tp.traces = (T *)H->traces;
            tp.nt_rec = H->nt_rec;
        }
        tp.ns = (int32_t)H->ns;
        tp.scells = H->d_src_cells;
        tp.sorder = H->d_src_order;
        tp.wav = (const T *)H->wavelets;
        tp.nt_src = H->nt_src;
        tp.amp = (T)(H->dt * H->dt / (H->h * H->h));
        tp.n = H->n;
    }
    // fork: the side stream starts once everything before this pass is done
    HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
    HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
    if (n_waves > 0) {
        dpmlk::StepArgs<T> p = make_args<T>(H);
        p.uout = nxt[0];
        p.tile_rows = rows;
        const dim3 grid((unsigned)round8((n_waves + 3) / 4), B);
        const int slot = timed_begin(H, DPML_KERNEL_PAIR, pass_bytes(H, core));
#define DPML_MULTI_LAUNCH(GG, C2)                                                                           \
        if (levels == 2)                                                                                    \
            hipLaunchKernelGGL((dpmlk::k_step2_march<T, VX, GG, C2>), grid, block, 0, H->stream, p, nxt[1],     \
                               r[0], r[1], r[2], r[3], strips, n_waves);                                    \
        else if (levels == 3)                                                                               \
            hipLaunchKernelGGL((dpmlk::k_step3_march<T, VX, GG, C2>), grid, block, 0, H->stream, p, nxt[1],     \
                               nxt[2], r[0], r[1], r[2], r[3], strips, n_waves);                            \
        else if (hist)                                                                                      \
            launch_coreN_hist<T>(levels, GG, C2, grid, H->stream, p, hist, hstride, nxt[levels - 2],          \
                                 nxt[levels - 1], r, strips, n_waves, tp);                                  \
        else                                                                                                \
            launch_coreN<T, VX, GG, C2>(levels, (H->tile_rows >> 24) & 1, grid, H->stream, p, nxt[levels - 2],    \
                                        nxt[levels - 1], r, strips, n_waves, tp);
        if (G == 4) {
            if (p.c2) { DPML_MULTI_LAUNCH(4, true) } else { DPML_MULTI_LAUNCH(4, false) }
        } else if (G == 1) {
            if (p.c2) { DPML_MULTI_LAUNCH(1, true) } else { DPML_MULTI_LAUNCH(1, false) }
        } else {
            if (p.c2) { DPML_MULTI_LAUNCH(2, true) } else { DPML_MULTI_LAUNCH(2, false) }
        }
#undef DPML_MULTI_LAUNCH
        timed_end(H, slot);
    }
    if (frame_fused(H)) {
        // all the frame's steps in one launch on the side stream; it reads the
        // aux buffer of level n and writes level n+levels to the other one
        const int nf = (int)H->n_ffused[q];
        if (nf > 0) {
            dpmlk::StepArgs<T> pj = make_args<T>(H);
            pj.u = A;
            pj.uo = Bv;
            for (int a = 0; a < 4; ++a) pj.skip[a] = r[a];
            const int slot = timed_begin(H, DPML_KERNEL_FRAME, levels * step_bytes(H, (double)L.ncell - core, aux_cells(L)),
                                         H->side);
            launch_fused<T>(levels, dim3((unsigned)round8(nf), B), H->side, pj, nxt[levels - 2], nxt[levels - 1],
                            H->d_ffused[q], nf);
            timed_end(H, slot, H->side);
        }
        HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
        HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
        HIP_TRY(H, hipGetLastError());
        H->u_now = nxt[levels - 1];
        H->u_old = nxt[levels - 2];
        H->cur = 1 - H->cur;
        H->n += levels;
        return DPML_OK;
    }
    // the frame's steps on the side stream: level j from level j-1 (U^n at
    // j = 1) and the level before it, aux buffers alternating
    for (int j = 1; j <= levels; ++j) {
        const int sh = levels - j;
        const int fr = frame_span_rows(H);
        const int nf = (int)(fr > 0 ? H->n_fspan[q][sh] : H->n_frame[q][sh]);
        if (nf <= 0) continue;
        if (j % 2 == 0) H->cur = 1 - H->cur;
        dpmlk::StepArgs<T> pj = make_args<T>(H);
        if (j % 2 == 0) H->cur = 1 - H->cur;
        pj.u = j == 1 ? A : nxt[j - 2];
        pj.uo = j == 1 ? Bv : (j == 2 ? A : nxt[j - 3]);
        pj.uout = nxt[j - 1];
        pj.skip[0] = r[0] + sh;
        pj.skip[1] = r[1] - sh;
        pj.skip[2] = r[2] + sh;
        pj.skip[3] = r[3] - sh;
        // algorithmic share: the frame's own cells (the ring cells it recomputes
        // are the core's, counted there)
        const int slot = timed_begin(H, DPML_KERNEL_FRAME, step_bytes(H, (double)L.ncell - core, aux_cells(L)), H->side);
        if (fr > 0)
            hipLaunchKernelGGL((dpmlk::k_step_frame_march<T, 4>), dim3((unsigned)round8((nf + 3) / 4), B), block, 0,
                               H->side, pj, H->d_fspan[q][sh], nf);
        else
            hipLaunchKernelGGL((dpmlk::k_step_frame<T>), dim3((unsigned)round8(nf), B), block, 0, H->side, pj,
                               H->d_frame[q][sh], nf);
        timed_end(H, slot, H->side);
        // the receivers less than levels-j cells inside the core, from this step's output
        const int64_t nrec = rec ? H->frec_count[q][j] : 0;
        if (nrec > 0 && H->n + j - 1 < H->nt_rec)
            hipLaunchKernelGGL((dpmlk::k_record_list<T>), dim3((unsigned)((nrec + 255) / 256)), block, 0, H->side,
                               (const T *)nxt[j - 1], H->d_frec_cells[q], H->d_frec_idx[q], nrec, (T *)H->traces,
                               H->nt_rec, H->n + j - 1);
    }
    // join
    HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
    HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
    HIP_TRY(H, hipGetLastError());
    H->u_now = nxt[levels - 1];
    H->u_old = nxt[levels - 2];
    if (levels % 2) H->cur = 1 - H->cur;
    H->n += levels;
    return DPML_OK;
}



template <typename T>
int step_impl(dpml *H, int64_t nsteps)
{
    int64_t k = 0;
    for (;;) {
        const int lv = multistep_levels(H, nsteps - k);
        if (lv < 2) break;
        int rc = ensure_multistep(H, lv);
        if (rc) return rc;
        rc = H->L.ndim == 3 ? launch_multistep3d<T>(H) : launch_multistep<T>(H, lv);
        if (rc) return rc;
        k += lv;
    }
    for (; k < nsteps; ++k) {
        int rc = launch_step<T>(H);
        if (rc) return rc;
        rc = launch_epilogue<T>(H);
        if (rc) return rc;
        std::swap(H->u_now, H->u_old);
        H->cur = 1 - H->cur;
        H->n += 1;
    }
    return DPML_OK;
}

template <typename T>
int set_state_impl(dpml *H, const void *U0, const void *V0)
{
    const Layout &L = H->L;
    H->u_now = H->at(L.off_u[0]);
    H->u_old = H->at(L.off_u[1]);
    H->cur = 0;
    HIP_TRY(H, hipMemcpyAsync(H->u_now, U0, (size_t)(L.ncell * L.batch) * sizeof(T), hipMemcpyDeviceToDevice, H->stream));
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        for (int k = 0; k < 2; ++k) {
            HIP_TRY(H, hipMemsetAsync(H->at(L.off_phi[a][k]), 0, (size_t)(L.aux_elems[a] * L.batch) * sizeof(T), H->stream));
            HIP_TRY(H, hipMemsetAsync(H->at(L.off_psi[a][k]), 0, (size_t)(L.aux_elems[a] * L.batch) * sizeof(T), H->stream));
        }
    }
    const T *c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
    const T inv_h2 = (T)(1.0 / (H->h * H->h));
    const T half_dt2 = (T)(0.5 * H->dt * H->dt);
    dim3 block(64, 4, 1);
    dim3 grid((unsigned)((L.N[0] + 63) / 64), (unsigned)((L.N[1] + 3) / 4),
              (unsigned)((L.ndim == 3 ? L.N[2] : 1) * L.batch));
    // read U0 from the caller's buffer (stream order puts the copy above first)
    if (L.ndim == 2)
        hipLaunchKernelGGL((dpmlk::k_start<T, 2>), grid, block, 0, H->stream, (const T *)U0, (const T *)V0,
                           (T *)H->u_old, c2, (T)H->c2_const, inv_h2, (T)H->dt, half_dt2,
                           (int)L.N[0], (int)L.N[1], (int)L.N[2], L.wall[0] | (L.wall[1] << 1) | (L.wall[2] << 2));
    else
        hipLaunchKernelGGL((dpmlk::k_start<T, 3>), grid, block, 0, H->stream, (const T *)U0, (const T *)V0,
                           (T *)H->u_old, c2, (T)H->c2_const, inv_h2, (T)H->dt, half_dt2,
                           (int)L.N[0], (int)L.N[1], (int)L.N[2], L.wall[0] | (L.wall[1] << 1) | (L.wall[2] << 2));
    HIP_TRY(H, hipGetLastError());
    H->n = 0;
    H->state_set = true;
    return DPML_OK;
}

template <typename T>
int upload_tables(dpml *H, const double *c2, int64_t c2_len, const double *const sigma[3])
{
    const Layout &L = H->L;
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        const int64_t N = L.N[a], b = L.lo[a] + L.n[a];
        std::vector<T> tab((size_t)L.M[a] + 1);
        for (int j = 0; j <= L.M[a]; ++j) {
            const int64_t i = (b + j) % N;
            tab[j] = sigma[a] ? (T)sigma[a][i] : T(0);
        }
        HIP_TRY(H, hipMemcpyAsync(H->at(L.off_sig[a]), tab.data(), tab.size() * sizeof(T),
                                  hipMemcpyHostToDevice, H->stream));
        HIP_TRY(H, hipStreamSynchronize(H->stream));
    }
    if (H->c2_field) {
        const int64_t chunk = (int64_t)1 << 24;
        std::vector<T> buf((size_t)std::min<int64_t>(chunk, L.ncell));
        for (int64_t s = 0; s < L.ncell; s += chunk) {
            const int64_t m = std::min(chunk, L.ncell - s);
            for (int64_t q = 0; q < m; ++q) buf[q] = (T)c2[s + q];
            HIP_TRY(H, hipMemcpyAsync((T *)H->at(L.off_c2) + s, buf.data(), (size_t)m * sizeof(T),
                                      hipMemcpyHostToDevice, H->stream));
            HIP_TRY(H, hipStreamSynchronize(H->stream));
        }
    }
    (void)c2_len;
    return DPML_OK;
}

// Is cell index i along axis a within one cell of the layer (or in it)?
bool near_layer(const Layout &L, int a, int64_t i)
{
    if (L.M[a] == 0) return false;
    return i >= L.lo[a] + L.n[a] - 1 || i <= L.lo[a];
}

// ---- allocation-free watchdog (dpml_step_checked_noalloc) ---------------
// Its scan flags live in this file-scope device array instead of the caller's
// workspace: one int32 flag per scan block.  Each GPU holds its own copy for
// the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device, looked
// up once at dpml_create), never through the array's name.
constexpr int kScratchFlags = 1024;
constexpr int64_t kMaxNoallocCells = (int64_t)1 << 40;   // the scan's 64-bit grid stride
static_assert(kScratchFlags >= kFlagBlocks, "the scan's flags must fit the static scratch");

}  // namespace

static __device__ __align__(256) int32_t scratch[kScratchFlags];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array (looked up once per device);
// nullptr with *err set on failure.
void *scratch_for_current_device(hipError_t *err)
{
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// The non-finite scan of U^n into the static flags: every scan block writes
// its flag, so nothing has to be cleared between calls.
template <typename T>
int nonfinite_check_noalloc(dpml *H, bool *bad)
{
    if (!H->scratch) return H->fail(DPML_EHIP, "no static scratch for this device");
    int32_t *flags = (int32_t *)H->scratch;
    hipLaunchKernelGGL((dpmlk::k_nonfinite<T>), dim3(kFlagBlocks), dim3(256), 0, H->stream,
                       (const T *)H->u_now, H->L.ncell * H->L.batch, flags);
    HIP_TRY(H, hipGetLastError());
    int32_t host[kFlagBlocks];
    HIP_TRY(H, hipMemcpyAsync(host, flags, sizeof(host), hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    *bad = false;
    for (int i = 0; i < kFlagBlocks; ++i) *bad |= host[i] != 0;
    return DPML_OK;
}

// One step by one thread per cell (no multi-step pass, no second stream, no
// table built on first use: nothing is allocated), sources and receivers
// from the tables registered beforehand.
template <typename T>
int step_cells_noalloc(dpml *H)
{
    const int variant = H->variant, rows = H->tile_rows;
    H->variant = DPML_VARIANT_CELL;
    H->tile_rows = 0;
    int rc = launch_step<T>(H);
    H->variant = variant;
    H->tile_rows = rows;
    if (rc) return rc;
    rc = launch_epilogue<T>(H);
    if (rc) return rc;
    std::swap(H->u_now, H->u_old);
    H->cur = 1 - H->cur;
    H->n += 1;
    return DPML_OK;
}

template <typename T>
int nonfinite_check(dpml *H, bool *bad)
{
    int32_t *flags = (int32_t *)H->at(H->L.off_flags);
    hipLaunchKernelGGL((dpmlk::k_nonfinite<T>), dim3(kFlagBlocks), dim3(256), 0, H->stream,
                       (const T *)H->u_now, H->L.ncell * H->L.batch, flags);
    HIP_TRY(H, hipGetLastError());
    std::vector<int32_t> host(kFlagBlocks);
    HIP_TRY(H, hipMemcpyAsync(host.data(), flags, kFlagBlocks * sizeof(int32_t), hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    *bad = std::any_of(host.begin(), host.end(), [](int32_t v) { return v != 0; });
    return DPML_OK;
}

}  // namespace

extern "C" {

size_t dpml_workspace_bytes(const dpml_grid_t *g, int32_t c2_is_field)
{
    Layout L;
    if (!make_layout(g, c2_is_field != 0, L, handle_ubufs(g)).empty()) return 0;
    return L.total;
}

int dpml_create(const dpml_grid_t *g, double h, double dt, const double *c2, int64_t c2_len,
                const double *const sigma[3], void *workspace, size_t ws_bytes, void *stream,
                dpml_t **out)
{
    if (!out) { g_create_error = "out is NULL"; return DPML_EINVAL; }
    *out = nullptr;
    Layout L;
    const bool field = c2_len != 1;
    std::string e = make_layout(g, field, L, handle_ubufs(g));
    if (!e.empty()) { g_create_error = e; return DPML_EINVAL; }
    if (!(h > 0) || !(dt > 0) || !std::isfinite(h) || !std::isfinite(dt)) {
        g_create_error = "h and dt must be positive and finite"; return DPML_EINVAL;
    }
    if (!c2 || (c2_len != 1 && c2_len != L.ncell)) {
        g_create_error = "c2 must hold 1 or prod(N) values"; return DPML_EINVAL;
    }
    // c^2 values: positive, finite, 1 on and next to the layer
    double c2max = 0;
    if (!field) {
        if (!(c2[0] > 0) || !std::isfinite(c2[0])) { g_create_error = "c2 must be positive and finite"; return DPML_EINVAL; }
        c2max = c2[0];
        bool any_layer = false;
        for (int a = 0; a < L.ndim; ++a) any_layer |= L.M[a] > 0;
        if (any_layer && c2[0] != 1.0) {
            g_create_error = "c2 must be 1 where damping acts (constant c2 != 1 with a layer)"; return DPML_EINVAL;
        }
    } else {
        for (int64_t c = 0; c < L.ncell; ++c) {
            const double v = c2[c];
            if (!(v > 0) || !std::isfinite(v)) { g_create_error = "c2 must be positive and finite"; return DPML_EINVAL; }
            c2max = std::max(c2max, v);
            if (v != 1.0) {
                const int64_t i[3] = {c % L.N[0], (c / L.N[0]) % L.N[1], c / (L.N[0] * L.N[1])};
                for (int a = 0; a < L.ndim; ++a)
                    if (near_layer(L, a, i[a])) {
                        g_create_error = "c2 must be 1 on the layer and within one cell of it";
                        return DPML_EINVAL;
                    }
            }
        }
    }
    if (std::sqrt(c2max) * dt / h * std::sqrt((double)L.ndim) > 1.0) {
        g_create_error = "time step violates c dt/h sqrt(ndim) <= 1"; return DPML_EINVAL;
    }
    double smax = 0;
    for (int a = 0; a < L.ndim; ++a) {
        if (!sigma || !sigma[a]) continue;
        for (int64_t i = 0; i < L.N[a]; ++i) {
            const double s = sigma[a][i];
            if (!(s >= 0) || !std::isfinite(s)) { g_create_error = "sigma must be >= 0 and finite"; return DPML_EINVAL; }
            if (s != 0 && i >= L.lo[a] && i < L.lo[a] + L.n[a]) {
                g_create_error = "sigma must vanish on the interior indices [lo, lo+n)"; return DPML_EINVAL;
            }
            smax = std::max(smax, s);
        }
    }
    if (dt * smax > 4.0) { g_create_error = "dt * max(sigma) must be <= 4"; return DPML_EINVAL; }
    if (!workspace || ws_bytes < L.total) {
        g_create_error = "workspace too small: need " + std::to_string(L.total) + " bytes";
        return DPML_ENOMEM;
    }
    if (((uintptr_t)workspace) % kAlign != 0) { g_create_error = "workspace must be 256-byte aligned"; return DPML_ENOMEM; }

    hipError_t serr = hipSuccess;
    void *sp = scratch_for_current_device(&serr);
    if (!sp) { g_create_error = std::string("static scratch lookup: ") + hipGetErrorString(serr); return DPML_EHIP; }
    dpml *H = new (std::nothrow) dpml();
    if (!H) { g_create_error = "out of host memory"; return DPML_ENOMEM; }
    H->scratch = sp;
    H->L = L;
    H->ws = (char *)workspace;
    H->stream = (hipStream_t)stream;
    H->h = h;
    H->dt = dt;
    H->c2_field = field;
    H->c2_const = field ? 1.0 : c2[0];
    const double *sig3[3] = {sigma ? sigma[0] : nullptr, sigma ? sigma[1] : nullptr,
                             sigma && L.ndim == 3 ? sigma[2] : nullptr};
    int rc = L.dtype == DPML_F32 ? upload_tables<float>(H, c2, c2_len, sig3)
                                 : upload_tables<double>(H, c2, c2_len, sig3);
    if (rc) { g_create_error = H->err; delete H; return rc; }
    *out = H;
    return DPML_OK;
}

int dpml_set_state(dpml_t *H, const void *U0, const void *V0)
{
    if (!H) return DPML_EINVAL;
    if (!U0) return H->fail(DPML_EINVAL, "U0 is NULL");
    return H->L.dtype == DPML_F32 ? set_state_impl<float>(H, U0, V0) : set_state_impl<double>(H, U0, V0);
}

int dpml_inject(dpml_t *H, int64_t ns, const int64_t *cells, const void *wavelets, int64_t nt)
{
    if (!H) return DPML_EINVAL;
    if (ns < 0 || (ns > 0 && (!cells || !wavelets || nt < 1))) return H->fail(DPML_EINVAL, "bad source arguments");
    for (int64_t s = 0; s < ns; ++s)
        if (cells[s] < 0 || cells[s] >= H->L.ncell * H->L.batch) return H->fail(DPML_EINVAL, "source cell out of range");
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    if (H->d_src_cells) { HIP_TRY(H, hipFree(H->d_src_cells)); H->d_src_cells = nullptr; }
    if (H->d_src_order) { HIP_TRY(H, hipFree(H->d_src_order)); H->d_src_order = nullptr; }
    H->ns = 0;
    H->src_sorted.clear();
    if (ns == 0) return DPML_OK;
    std::vector<int64_t> order((size_t)ns);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cells[a] < cells[b]; });
    std::vector<int64_t> sorted((size_t)ns);
    for (int64_t q = 0; q < ns; ++q) sorted[q] = cells[order[q]];
    HIP_TRY(H, hipMalloc((void **)&H->d_src_cells, (size_t)ns * sizeof(int64_t)));
    HIP_TRY(H, hipMalloc((void **)&H->d_src_order, (size_t)ns * sizeof(int64_t)));
    HIP_TRY(H, hipMemcpy(H->d_src_cells, sorted.data(), (size_t)ns * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(H, hipMemcpy(H->d_src_order, order.data(), (size_t)ns * sizeof(int64_t), hipMemcpyHostToDevice));
    H->ns = ns;
    H->nt_src = nt;
    H->wavelets = wavelets;
    H->src_sorted = sorted;
    return DPML_OK;
}

int dpml_record(dpml_t *H, int64_t nr, const int64_t *cells, void *traces, int64_t nt)
{
    if (!H) return DPML_EINVAL;
    if (nr < 0 || (nr > 0 && (!cells || !traces || nt < 1))) return H->fail(DPML_EINVAL, "bad receiver arguments");
    for (int64_t r = 0; r < nr; ++r)
        if (cells[r] < 0 || cells[r] >= H->L.ncell * H->L.batch) return H->fail(DPML_EINVAL, "receiver cell out of range");
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    for (int64_t **pp : {&H->d_rec_cells, &H->d_rec_sorted, &H->d_rec_order})
        if (*pp) { HIP_TRY(H, hipFree(*pp)); *pp = nullptr; }
    free_taps(H);
    H->rec_host.assign(cells, cells + nr);
    H->nr = 0;
    if (nr == 0) return DPML_OK;
    std::vector<int64_t> order((size_t)nr);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cells[a] < cells[b]; });
    std::vector<int64_t> sorted((size_t)nr);
    for (int64_t q = 0; q < nr; ++q) sorted[q] = cells[order[q]];
    H->rec_dups = false;
    for (int64_t q = 1; q < nr; ++q) H->rec_dups |= sorted[q] == sorted[q - 1];
    HIP_TRY(H, hipMalloc((void **)&H->d_rec_cells, (size_t)nr * sizeof(int64_t)));
    HIP_TRY(H, hipMalloc((void **)&H->d_rec_sorted, (size_t)nr * sizeof(int64_t)));
    HIP_TRY(H, hipMalloc((void **)&H->d_rec_order, (size_t)nr * sizeof(int64_t)));
    HIP_TRY(H, hipMemcpy(H->d_rec_cells, cells, (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(H, hipMemcpy(H->d_rec_sorted, sorted.data(), (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(H, hipMemcpy(H->d_rec_order, order.data(), (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice));
    H->nr = nr;
    H->nt_rec = nt;
    H->traces = traces;
    return DPML_OK;
}

int dpml_record_plane(dpml_t *H, int32_t axis, int64_t index, void *planes, int64_t nt)
{
    if (!H) return DPML_EINVAL;
    if (axis < 0) { H->plane_axis = -1; return DPML_OK; }
    if (axis >= H->L.ndim || index < 0 || index >= H->L.N[axis] || !planes || nt < 1 || H->L.batch != 1)
        return H->fail(DPML_EINVAL, "bad plane recorder arguments");
    H->plane_axis = axis;
    H->plane_index = index;
    H->planes = planes;
    H->nt_plane = nt;
    return DPML_OK;
}

int dpml_set_variant(dpml_t *H, int32_t variant, int32_t tile_rows)
{
    if (!H) return DPML_EINVAL;
    // highest shape bit + 1: 3D multi-step passes read bits up to 30, 3D MARCH
    // up to 29, DEEP up to 24, the others up to 19
    const bool d3 = H->L.ndim == 3;
    const int bits = variant == DPML_VARIANT_DEEP ? 25
                     : (d3 && variant >= DPML_VARIANT_TWOSTEP) ? 31
                     : (d3 && variant == DPML_VARIANT_MARCH) ? 30 : 20;
    if (variant < DPML_VARIANT_AUTO || variant > DPML_VARIANT_DEEP || tile_rows < 0 ||
        (bits < 31 && tile_rows >= (1 << bits)))
        return H->fail(DPML_EINVAL, "bad variant");
    if (variant == DPML_VARIANT_DEEP && (pass_depth(variant, tile_rows) < 2 || pass_depth(variant, tile_rows) > kMaxLevels))
        return H->fail(DPML_EINVAL, "DEEP passes take 2 .. 8 levels");
    H->variant = variant;
    H->tile_rows = tile_rows;
    return DPML_OK;
}

int dpml_step(dpml_t *H, int64_t nsteps)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0) return H->fail(DPML_EINVAL, "nsteps < 0");
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    return H->L.dtype == DPML_F32 ? step_impl<float>(H, nsteps) : step_impl<double>(H, nsteps);
}

int dpml_step_checked(dpml_t *H, int64_t nsteps, int64_t every)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0 || every < 1) return H->fail(DPML_EINVAL, "nsteps < 0 or every < 1");
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t k = std::min(every, nsteps - done);
        int rc = dpml_step(H, k);
        if (rc) return rc;
        done += k;
        bool bad = false;
        rc = H->L.dtype == DPML_F32 ? nonfinite_check<float>(H, &bad) : nonfinite_check<double>(H, &bad);
        if (rc) return rc;
        if (bad) return H->fail(DPML_ENONFINITE, "non-finite value in U at step " + std::to_string(H->n));
    }
    return DPML_OK;
}

int dpml_step_checked_noalloc(dpml_t *H, int64_t nsteps, int64_t every)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0 || every < 1) return H->fail(DPML_EINVAL, "nsteps < 0 or every < 1");
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    if (H->L.ncell * H->L.batch > kMaxNoallocCells)
        return H->fail(DPML_EINVAL, "grid larger than the allocation-free scan handles (2^40 cells)");
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t k = std::min(every, nsteps - done);
        for (int64_t i = 0; i < k; ++i) {
            int rc = H->L.dtype == DPML_F32 ? step_cells_noalloc<float>(H) : step_cells_noalloc<double>(H);
            if (rc) return rc;
        }
        done += k;
        bool bad = false;
        int rc = H->L.dtype == DPML_F32 ? nonfinite_check_noalloc<float>(H, &bad)
                                        : nonfinite_check_noalloc<double>(H, &bad);
        if (rc) return rc;
        if (bad) return H->fail(DPML_ENONFINITE, "non-finite value in U at step " + std::to_string(H->n));
    }
    return DPML_OK;
}

int dpml_field(dpml_t *H, int32_t which, void **ptr, int64_t shape[3])
{
    if (!H || !ptr || !shape) return DPML_EINVAL;
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    const Layout &L = H->L;
    for (int a = 0; a < 3; ++a) shape[a] = L.N[a];
    if (which == DPML_FIELD_U) { *ptr = H->u_now; return DPML_OK; }
    if (which == DPML_FIELD_UPREV) { *ptr = H->u_old; return DPML_OK; }
    const int a = (which - 2) / 2;
    if (which < 2 || a >= L.ndim || L.M[a] == 0) return H->fail(DPML_EINVAL, "no such field");
    shape[a] = L.M[a] + 1;
    *ptr = H->at((which % 2 == 0) ? L.off_phi[a][H->cur] : L.off_psi[a][H->cur]);
    return DPML_OK;
}

int64_t dpml_time_index(const dpml_t *H) { return H ? H->n : -1; }

size_t dpml_state_bytes(const dpml_t *H)
{
    if (!H) return 0;
    const Layout &L = H->L;
    size_t b = 2 * (size_t)(L.ncell * L.batch) * L.esize;
    for (int a = 0; a < L.ndim; ++a) b += 2 * (size_t)(L.aux_elems[a] * L.batch) * L.esize;
    return b;
}

namespace {
// Copy the state between the handle and a blob; to_blob selects the direction.
int copy_state(dpml_t *H, char *blob, bool to_blob)
{
    const Layout &L = H->L;
    size_t off = 0;
    auto cp = [&](void *dev, size_t bytes) -> int {
        void *dst = to_blob ? (void *)(blob + off) : dev;
        const void *src = to_blob ? (const void *)dev : (const void *)(blob + off);
        HIP_TRY(H, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, H->stream));
        off += bytes;
        return DPML_OK;
    };
    const size_t ub = (size_t)(L.ncell * L.batch) * L.esize;
    int rc = cp(H->u_now, ub);
    if (!rc) rc = cp(H->u_old, ub);
    for (int a = 0; a < L.ndim && !rc; ++a) {
        if (L.M[a] == 0) continue;
        const size_t ab = (size_t)(L.aux_elems[a] * L.batch) * L.esize;
        rc = cp(H->at(L.off_phi[a][H->cur]), ab);
        if (!rc) rc = cp(H->at(L.off_psi[a][H->cur]), ab);
    }
    return rc;
}
}  // namespace

int dpml_get_state(dpml_t *H, void *blob)
{
    if (!H || !blob) return DPML_EINVAL;
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    return copy_state(H, (char *)blob, true);
}

int dpml_put_state(dpml_t *H, const void *blob, int64_t n)
{
    if (!H || !blob || n < 0) return DPML_EINVAL;
    const Layout &L = H->L;
    if (!H->state_set) {
        H->u_now = H->at(L.off_u[0]);
        H->u_old = H->at(L.off_u[1]);
        H->cur = 0;
        // the spare aux buffers must hold zeros in the slots no step writes
        for (int a = 0; a < L.ndim; ++a) {
            if (L.M[a] == 0) continue;
            for (int k = 0; k < 2; ++k) {
                HIP_TRY(H, hipMemsetAsync(H->at(L.off_phi[a][k]), 0, (size_t)(L.aux_elems[a] * L.batch) * L.esize, H->stream));
                HIP_TRY(H, hipMemsetAsync(H->at(L.off_psi[a][k]), 0, (size_t)(L.aux_elems[a] * L.batch) * L.esize, H->stream));
            }
        }
    }
    int rc = copy_state(H, (char *)blob, false);
    if (rc) return rc;
    H->n = n;
    H->state_set = true;
    return DPML_OK;
}

int dpml_sync(dpml_t *H)
{
    if (!H) return DPML_EINVAL;
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}

int dpml_set_timing(dpml_t *H, int32_t enable)
{
    if (!H) return DPML_EINVAL;
    if (enable && !H->timing) {
        H->timed.clear();
        H->events_used = 0;
    }
    H->timing = enable != 0;
    return DPML_OK;
}

int dpml_get_timing(dpml_t *H, dpml_timing_t *out)
{
    if (!H || !out) return DPML_EINVAL;
    *out = dpml_timing_t{};
    for (const dpml::Timed &t : H->timed) HIP_TRY(H, hipEventSynchronize(t.e1));
    for (const dpml::Timed &t : H->timed) {
        float ms = 0.f;
        HIP_TRY(H, hipEventElapsedTime(&ms, t.e0, t.e1));
        out->launches[t.kind] += 1;
        out->ms[t.kind] += ms;
        out->bytes[t.kind] += t.bytes;
    }
    H->timed.clear();
    H->events_used = 0;
    return DPML_OK;
}

void dpml_destroy(dpml_t *H)
{
    if (!H) return;
    (void)hipStreamSynchronize(H->stream);
    if (H->exec) (void)hipGraphExecDestroy(H->exec);
    if (H->graph) (void)hipGraphDestroy(H->graph);
    if (H->cap) (void)hipStreamDestroy(H->cap);
    if (H->d_src_cells) (void)hipFree(H->d_src_cells);
    if (H->d_src_order) (void)hipFree(H->d_src_order);
    if (H->d_rec_cells) (void)hipFree(H->d_rec_cells);
    for (int k = 0; k < kMaxLevels - 1; ++k)
        for (int j = 0; j < kMaxLevels; ++j) {
            if (H->d_frame[k][j]) (void)hipFree(H->d_frame[k][j]);
            if (H->d_fspan[k][j]) (void)hipFree(H->d_fspan[k][j]);
        }
    for (int k = 0; k < kMaxLevels - 1; ++k)
        if (H->d_ffused[k]) (void)hipFree(H->d_ffused[k]);
    if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
    if (H->ev_join) (void)hipEventDestroy(H->ev_join);
    if (H->side) (void)hipStreamDestroy(H->side);
    for (hipEvent_t e : {H->adj_rfork, H->adj_rjoin, H->adj_rec_done[0], H->adj_rec_done[1], H->adj_sweep_done[0],
                         H->adj_sweep_done[1]})
        if (e) (void)hipEventDestroy(e);
    if (H->adj_rside) (void)hipStreamDestroy(H->adj_rside);
    if (H->adj_rs) (void)hipStreamDestroy(H->adj_rs);
    if (H->d_adj_frame) (void)hipFree(H->d_adj_frame);
    for (int k = 0; k < 2; ++k)
        if (H->d_adj_frame_s[k]) (void)hipFree(H->d_adj_frame_s[k]);
    free_taps(H);
    if (H->d_rec_sorted) (void)hipFree(H->d_rec_sorted);
    if (H->d_rec_order) (void)hipFree(H->d_rec_order);
    for (hipEvent_t e : H->events) (void)hipEventDestroy(e);
    delete H;
}

const char *dpml_strerror(int code)
{
    switch (code) {
    case DPML_OK: return "ok";
    case DPML_EINVAL: return "invalid argument";
    case DPML_ENOMEM: return "insufficient memory or workspace";
    case DPML_EHIP: return "HIP runtime error";
    case DPML_ESTATE: return "invalid state for this call";
    case DPML_ENONFINITE: return "non-finite value in the wave field";
    default: return "unknown error";
    }
}

const char *dpml_last_error(const dpml_t *H)
{
    return H ? H->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpointed forward and discrete adjoint
// ---------------------------------------------------------------------------
namespace {

struct AdjLayout {
    int64_t nck = 0;
    size_t state = 0, off_ckpt = 0, level = 0, off_hist[2] = {0, 0};
    size_t off_lam[4] = {0, 0, 0, 0};
    size_t off_p[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t off_q[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t total = 0;
};

AdjLayout adj_layout(const dpml *H, int64_t nsteps, int64_t every)
{
    const Layout &L = H->L;
    AdjLayout A;
    A.nck = (nsteps + every - 1) / every;
    A.state = align_up(dpml_state_bytes(H));
    A.level = align_up((size_t)(L.ncell * L.batch) * L.esize);
    size_t off = 0;
    A.off_ckpt = off; off += (size_t)A.nck * A.state;
    // two segments' histories: the next segment's recompute fills one while
    // the reverse sweep reads the other
    for (int k = 0; k < 2; ++k) { A.off_hist[k] = off; off += (size_t)every * A.level; }
    for (int k = 0; k < 4; ++k) { A.off_lam[k] = off; off += A.level; }
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        const size_t ab = align_up((size_t)(L.aux_elems[a] * L.batch) * L.esize);
        for (int k = 0; k < 2; ++k) {
            A.off_p[a][k] = off; off += ab;
            A.off_q[a][k] = off; off += ab;
        }
    }
    A.total = off;
    return A;
}

template <typename T>
int forward_ckpt_impl(dpml *H, int64_t nsteps)
{
    const AdjLayout A = adj_layout(H, nsteps, H->adj_every);
    // a checkpoint every adj_every steps; the steps between two checkpoints
    // go as one run (multi-step passes where the variant takes them)
    for (int64_t k = 0; k < nsteps;) {
        if (k % H->adj_every == 0) {
            int rc = copy_state(H, H->adj_ws + A.off_ckpt + (size_t)(k / H->adj_every) * A.state, true);
            if (rc) return rc;
        }
        const int64_t seg = std::min(H->adj_every - k % H->adj_every, nsteps - k);
        int rc = step_impl<T>(H, seg);
        if (rc) return rc;
        k += seg;
    }
    return DPML_OK;
}

constexpr int kAdjRows = 4;   // rows per wave of the 2D marching adjoint kernel
constexpr int kAdjFrameGroups = 8;   // waves (shot groups) per block of the 2D adjoint frame
constexpr int kAdjFrameGroupsBuf = 4;   // ... in its buffer-descriptor form (fewer registers: more blocks per CU)
template <typename T>
constexpr int kAdjFrameShots = sizeof(T) == 4 ? 2 : 1;   // shots whose loads a frame wave issues together

// Core of the 2D adjoint: cells whose update, and whose neighbours' band
// slots, carry no layer term: [lo+2, lo+n-1) on an axis with a layer, the
// whole axis without one.  Returns {x0, x1, y0, y1}.
void adj_core(const Layout &L, int r[4])
{
    for (int a = 0; a < 2; ++a) {
        if (L.M[a] == 0) {
            r[2 * a] = 0;
            r[2 * a + 1] = (int)L.N[a];
        } else {
            r[2 * a] = L.lo[a] + 2;
            r[2 * a + 1] = std::max(r[2 * a], (int)(L.lo[a] + L.n[a] - 1));
        }
    }
}

// The adjoint core shrunk by s cells on every axis with a layer (an axis
// without one stays whole: it has no frame).
void adj_core_shrunk(const Layout &L, int s, int r[4])
{
    adj_core(L, r);
    for (int a = 0; a < 2; ++a) {
        if (L.M[a] == 0) continue;
        r[2 * a] += s;
        r[2 * a + 1] = std::max(r[2 * a], r[2 * a + 1] - s);
    }
}

// 64 x 4 tiles holding any cell outside the adjoint core shrunk by s (0, 1
// or 2): the frame of a single step, and of the two steps of a two-level
// pass.
int ensure_adj_frame(dpml *H, int s = 0)
{
    dpmlk::TileRef **dst = s == 0 ? &H->d_adj_frame : &H->d_adj_frame_s[s - 1];
    int64_t *cnt = s == 0 ? &H->n_adj_frame : &H->n_adj_frame_s[s - 1];
    if (*cnt >= 0) return DPML_OK;
    const Layout &L = H->L;
    int r[4];
    adj_core_shrunk(L, s, r);
    std::vector<dpmlk::TileRef> t;
    const int tx = (int)((L.N[0] + 63) / 64), ty = (int)((L.N[1] + 3) / 4);
    for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x) {
            const int xa = x * 64, xb = std::min<int>(xa + 64, (int)L.N[0]);
            const int ya = y * 4, yb = std::min<int>(ya + 4, (int)L.N[1]);
            if (!(xa >= r[0] && xb <= r[1] && ya >= r[2] && yb <= r[3])) t.push_back({0, x, y, 0});
        }
    *cnt = (int64_t)t.size();
    if (t.empty()) return DPML_OK;
    HIP_TRY(H, hipMalloc((void **)dst, t.size() * sizeof(dpmlk::TileRef)));
    HIP_TRY(H, hipMemcpy(*dst, t.data(), t.size() * sizeof(dpmlk::TileRef), hipMemcpyHostToDevice));
    return DPML_OK;
}

// The receivers outside rectangle S (the cells whose a^n the frame's first
// step of a two-level pass writes), sorted by cell, with their indices.
int ensure_adj_frec(dpml *H, const int S[4])
{
    if (H->n_adj_frec >= 0) return DPML_OK;
    const Layout &L = H->L;
    const int NX = (int)L.N[0];
    std::vector<std::pair<int64_t, int64_t>> v;
    for (int64_t i = 0; i < (int64_t)H->rec_host.size(); ++i) {
        const int64_t c = H->rec_host[i] % L.ncell;
        const int x = (int)(c % NX), y = (int)(c / NX);
        if (!(x >= S[0] && x < S[1] && y >= S[2] && y < S[3])) v.push_back({H->rec_host[i], i});
    }
    std::sort(v.begin(), v.end());
    H->n_adj_frec = (int64_t)v.size();
    if (v.empty()) return DPML_OK;
    std::vector<int64_t> cells(v.size()), order(v.size());
    for (size_t k = 0; k < v.size(); ++k) {
        cells[k] = v[k].first;
        order[k] = v[k].second;
    }
    HIP_TRY(H, hipMalloc((void **)&H->d_adj_frec_cells, v.size() * sizeof(int64_t)));
    HIP_TRY(H, hipMalloc((void **)&H->d_adj_frec_order, v.size() * sizeof(int64_t)));
    HIP_TRY(H, hipMemcpy(H->d_adj_frec_cells, cells.data(), v.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(H, hipMemcpy(H->d_adj_frec_order, order.data(), v.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    return DPML_OK;
}

template <typename T>
int adjoint_impl(dpml *H, const void *resid, double *grad, void *grad_w)
{
    const Layout &L = H->L;
    const int64_t nsteps = H->adj_nsteps, every = H->adj_every;
    const AdjLayout A = adj_layout(H, nsteps, every);
    char *ws = H->adj_ws;
    const size_t lb = (size_t)(L.ncell * L.batch) * sizeof(T);
    // the recompute's streams and the events that order it against the sweep
    if (!H->adj_rs) HIP_TRY(H, hipStreamCreateWithFlags(&H->adj_rs, hipStreamNonBlocking));
    if (!H->adj_rside) HIP_TRY(H, hipStreamCreateWithFlags(&H->adj_rside, hipStreamNonBlocking));
    for (hipEvent_t *e : {&H->adj_rfork, &H->adj_rjoin, &H->adj_rec_done[0], &H->adj_rec_done[1],
                          &H->adj_sweep_done[0], &H->adj_sweep_done[1]})
        if (!*e) HIP_TRY(H, hipEventCreateWithFlags(e, hipEventDisableTiming));
    for (int k = 0; k < 4; ++k) HIP_TRY(H, hipMemsetAsync(ws + A.off_lam[k], 0, lb, H->stream));
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        const size_t ab = (size_t)(L.aux_elems[a] * L.batch) * sizeof(T);
        for (int k = 0; k < 2; ++k) {
            HIP_TRY(H, hipMemsetAsync(ws + A.off_p[a][k], 0, ab, H->stream));
            HIP_TRY(H, hipMemsetAsync(ws + A.off_q[a][k], 0, ab, H->stream));
        }
    }
    int il = 0, io = 1;   // lam[il] = a^{n+1}, lam[io] = a^{n+2}; the other two take a two-level pass's output
    int acur = 0;         // p/q[acur] = adjoint auxiliaries at level n+1
    double hd = 1;
    for (int a = 0; a < L.ndim; ++a) hd *= H->h;
    const T wamp = (T)(H->dt * H->dt / hd);
    H->recording = false;
    dim3 block(64, 4, 1);
    dim3 grid((unsigned)((L.N[0] + 63) / 64), (unsigned)((L.N[1] + 3) / 4), (unsigned)(L.ndim == 3 ? L.N[2] : 1));
    const int adj_tiles = (int)(((L.N[0] + 63) / 64) * ((L.N[1] + 3) / 4) * (L.ndim == 3 ? L.N[2] : 1));
    const dim3 agrid((unsigned)round8(adj_tiles)), ablock(256);
    // 2D: the core in marching waves of 64 columns x kAdjRows rows, the
    // frame one thread per cell over a tile list
    int core[4] = {0, 0, 0, 0};
    int adj_tiles_x = 0, adj_waves = 0;
    // the frame kernel addresses a member's field and each axis's compact
    // auxiliaries by 32-bit byte offsets: larger 2D members take one thread
    // per cell over the whole grid
    bool fits32 = (uint64_t)L.ncell * L.esize < (1ull << 32);
    for (int a = 0; a < L.ndim; ++a) fits32 &= (uint64_t)L.aux_elems[a] * L.esize < (1ull << 32);
    const bool march2d = L.ndim == 2 && fits32;
    // the frame's buffer descriptors span all members of an array
    bool frame_buf = (uint64_t)L.batch * L.ncell * L.esize < (1ull << 32);
    for (int a = 0; a < L.ndim; ++a) frame_buf &= (uint64_t)L.batch * L.aux_elems[a] * L.esize < (1ull << 32);
    if (march2d) {
        int rc = ensure_adj_frame(H);
        if (!rc) rc = ensure_side(H);
        if (rc) return rc;
        adj_core(L, core);
        adj_tiles_x = (core[1] - core[0] + 63) / 64;
        adj_waves = adj_tiles_x * ((core[3] - core[2] + kAdjRows - 1) / kAdjRows);
    }
    // two-level passes (2D): a core r = the adjoint core shrunk by one, a^n
    // stored on r shrunk by one (core2s), the frame's two steps outside those;
    // receivers on distinct cells (the core adds the residual of the second
    // step in registers)
    int core2[4] = {0, 0, 0, 0}, core2s[4] = {0, 0, 0, 0};
    int tiles2_x = 0, waves2 = 0;
    bool two_ok = false;
    if (march2d) {
        adj_core_shrunk(L, 1, core2);
        adj_core_shrunk(L, 2, core2s);
        if (core2[1] > core2[0] && core2[3] > core2[2] && !(H->nr > 0 && H->rec_dups)) {
            int rc = ensure_adj_frame(H, 1);
            if (!rc) rc = ensure_adj_frame(H, 2);
            if (!rc && H->nr > 0) rc = ensure_rmap(H);
            if (!rc && H->nr > 0) rc = ensure_adj_frec(H, core2s);
            if (rc) return rc;
            tiles2_x = (core2[1] - core2[0] + 61) / 62;
            waves2 = tiles2_x * ((core2[3] - core2[2] + kAdjRows - 1) / kAdjRows);
            two_ok = true;
        }
    }
    const dim3 mgrid((unsigned)round8((adj_waves + 3) / 4));
    // The recompute of a segment: restore its checkpoint and recompute U^{t0}
    // .. U^{t1-1} into the segment's history buffer (seg & 1).  U^{t0} goes to
    // slot 0; each recomputed level is then written straight into its slot:
    // the multi-step passes keep every level they form (the levels the
    // handle's variant takes, 2 or 4 and more), the rest single steps reading
    // the two previous slots.  It runs on the recompute's own streams, so the
    // next segment's recompute overlaps the current segment's reverse sweep;
    // the sweep of a segment waits for its recompute, and a recompute waits
    // for the sweep that last read its history buffer.
    const int64_t hstride = (int64_t)(A.level / sizeof(T));
    auto recompute_body = [&](int64_t seg) -> int {
        const int64_t t0 = seg * every, t1 = std::min(t0 + every, nsteps);
        char *hist = ws + A.off_hist[seg & 1];
        H->state_set = true;
        H->cur = 0;
        H->u_now = H->at(L.off_u[0]);
        H->u_old = H->at(L.off_u[1]);
        int rc = copy_state(H, ws + A.off_ckpt + (size_t)seg * A.state, false);
        if (rc) return rc;
        H->n = t0;
        HIP_TRY(H, hipMemcpyAsync(hist, H->u_now, lb, hipMemcpyDeviceToDevice, H->stream));
        H->u_now = hist;
        for (int64_t k = t0; k + 1 < t1;) {
            T *slot = (T *)(hist + (size_t)(k - t0 + 1) * A.level);
            int lv = L.ndim == 2 ? multistep_levels(H, t1 - 1 - k) : 1;
            if (lv == 3) lv = 2;
            if (lv >= 2 && frame_fused(H)) lv = 1;
            if (lv >= 2) {
                rc = ensure_multistep(H, lv);
                if (!rc) rc = launch_multistep<T>(H, lv, slot, hstride);
                if (rc) return rc;
                k += lv;
                continue;
            }
            T *cur = (T *)H->u_now;         // U^k; u_old holds U^{k-1}
            rc = launch_step<T>(H, nullptr, slot);
            if (rc) return rc;
            if (H->ns > 0 && H->n < H->nt_src) {
                dim3 g2((unsigned)((H->ns + 255) / 256)), b2(256);
                hipLaunchKernelGGL((dpmlk::k_inject<T>), g2, b2, 0, H->stream, slot, H->d_src_cells,
                                   H->d_src_order, (const T *)H->wavelets, H->ns, H->nt_src, H->n, wamp);
            }
            H->u_old = cur;
            H->u_now = slot;
            H->cur = 1 - H->cur;
            H->n += 1;
            ++k;
        }
        HIP_TRY(H, hipEventRecord(H->adj_rec_done[seg & 1], H->stream));
        return DPML_OK;
    };
    // enqueue a recompute with the recompute's streams and events standing in
    // for the handle's own (every launch path takes those four)
    auto recompute = [&](int64_t seg) -> int {
        std::swap(H->stream, H->adj_rs);
        std::swap(H->side, H->adj_rside);
        std::swap(H->ev_fork, H->adj_rfork);
        std::swap(H->ev_join, H->adj_rjoin);
        const int rc = recompute_body(seg);
        std::swap(H->stream, H->adj_rs);
        std::swap(H->side, H->adj_rside);
        std::swap(H->ev_fork, H->adj_rfork);
        std::swap(H->ev_join, H->adj_rjoin);
        return rc;
    };
    {
        // the recompute stream starts after everything enqueued before this call
        HIP_TRY(H, hipEventRecord(H->adj_sweep_done[0], H->stream));
        HIP_TRY(H, hipStreamWaitEvent(H->adj_rs, H->adj_sweep_done[0], 0));
        const int rc = recompute(A.nck - 1);
        if (rc) return rc;
    }
    for (int64_t seg = A.nck - 1; seg >= 0; --seg) {
        const int64_t t0 = seg * every, t1 = std::min(t0 + every, nsteps);
        const char *hist = ws + A.off_hist[seg & 1];
        HIP_TRY(H, hipStreamWaitEvent(H->stream, H->adj_rec_done[seg & 1], 0));
        if (seg > 0) {
            // the previous segment's recompute refills the buffer the sweep of
            // segment seg + 1 read
            if (seg + 1 < A.nck) HIP_TRY(H, hipStreamWaitEvent(H->adj_rs, H->adj_sweep_done[(seg + 1) & 1], 0));
            const int rc = recompute(seg - 1);
            if (rc) return rc;
        }
        // reverse sweep over the segment
        auto lamb = [&](int k) { return (T *)(ws + A.off_lam[k]); };
        // arguments of the transposed step n (adjoint auxiliaries at n+1 in p/q[ai])
        auto base = [&](int64_t n, int ai) {
            dpmlk::AdjArgs<T> q{};
            for (int a = 0; a < 3; ++a) {
                q.ax[a] = make_axis<T>(H, a, false);
                if (a < L.ndim && L.M[a] > 0) {
                    q.ax[a].phi = (const T *)(ws + A.off_p[a][ai]);
                    q.ax[a].psi = (const T *)(ws + A.off_q[a][ai]);
                    q.ax[a].phi_o = (T *)(ws + A.off_p[a][1 - ai]);
                    q.ax[a].psi_o = (T *)(ws + A.off_q[a][1 - ai]);
                }
                q.bstride_aux[a] = L.aux_elems[a];
            }
            q.un = (const T *)(hist + (size_t)(n - t0) * A.level);
            q.c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
            q.grad = grad;
            q.c2_const = (T)H->c2_const;
            q.inv_h2 = (T)(1.0 / (H->h * H->h));
            q.inv_2h = (T)(1.0 / (2.0 * H->h));
            q.dt = (T)H->dt;
            q.dt2 = (T)(H->dt * H->dt);
            q.half_dt = (T)(0.5 * H->dt);
            q.k_damp = (T)(H->dt * H->dt / H->h);
            q.nx = (int32_t)L.N[0];
            q.ny = (int32_t)L.N[1];
            q.nz = (int32_t)L.N[2];
            q.batch = (int32_t)L.batch;
            q.bstride = L.ncell;
            return q;
        };
        // the residual of step n into a^{n+1}
        auto inject = [&](T *dst, int64_t n, hipStream_t st) {
            if (H->nr > 0 && n < H->nt_rec) {
                dim3 g2((unsigned)((H->nr + 255) / 256)), b2(256);
                hipLaunchKernelGGL((dpmlk::k_inject<T>), g2, b2, 0, st, dst, H->d_rec_sorted, H->d_rec_order,
                                   (const T *)resid, H->nr, H->nt_rec, n, (T)1);
            }
        };
        // dJ/dw of step n from a^{n+1} (nothing writes a^{n+1} while the step runs)
        auto gather = [&](const T *src, int64_t n, hipStream_t st) {
            if (H->ns > 0 && n < H->nt_src && grad_w) {
                dim3 g2((unsigned)((H->ns + 255) / 256)), b2(256);
                hipLaunchKernelGGL((dpmlk::k_gather_scaled<T>), g2, b2, 0, st, src, H->d_src_cells,
                                   H->d_src_order, (T *)grad_w, H->ns, H->nt_src, n, wamp);
            }
        };
        auto frame = [&](dpmlk::AdjArgs<T> f, const dpmlk::TileRef *tiles, int64_t nt, const int skip[4],
                         const int gskip[4], hipStream_t st) {
            if (nt <= 0) return;
            f.tiles = tiles;
            f.ntiles = (int32_t)nt;
            for (int k = 0; k < 4; ++k) {
                f.skip[k] = skip[k];
                f.gskip[k] = gskip[k];
            }
            if (frame_buf)
                hipLaunchKernelGGL((dpmlk::k_adjoint_frame2d<T, kAdjFrameGroupsBuf, kAdjFrameShots<T>, true>),
                                   dim3((unsigned)round8(4 * (int)nt)), dim3(64 * kAdjFrameGroupsBuf), 0, st, f);
            else
                hipLaunchKernelGGL((dpmlk::k_adjoint_frame2d<T, kAdjFrameGroups, kAdjFrameShots<T>, false>),
                                   dim3((unsigned)round8(4 * (int)nt)), dim3(64 * kAdjFrameGroups), 0, st, f);
        };
        const int none[4] = {0, 0, 0, 0};
        for (int64_t n = t1 - 1; n >= t0;) {
            T *lam = lamb(il), *lam_o = lamb(io);
            inject(lam, n, H->stream);
            if (two_ok && n - 1 >= t0) {
                // steps n and n-1 in one pass: the core both in registers, the
                // frame's two single steps beside it on the side stream
                int fr[2], nf = 0;
                for (int k = 0; k < 4; ++k)
                    if (k != il && k != io) fr[nf++] = k;
                T *out1 = lamb(fr[0]), *out2 = lamb(fr[1]);
                HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
                HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
                gather(lam, n, H->side);
                {
                    // step n outside core2s (its gradient only outside core2: the core adds the ring's)
                    dpmlk::AdjArgs<T> f = base(n, acur);
                    f.lam = lam;
                    f.lam_o = lam_o;
                    f.lam_w = out1;
                    frame(f, H->d_adj_frame_s[1], H->n_adj_frame_s[1], core2s, core2, H->side);
                }
                // the residual of step n-1 at the receivers whose a^n the frame wrote
                if (H->nr > 0 && n - 1 < H->nt_rec && H->n_adj_frec > 0) {
                    dim3 g2((unsigned)((H->n_adj_frec + 255) / 256)), b2(256);
                    hipLaunchKernelGGL((dpmlk::k_inject<T>), g2, b2, 0, H->side, out1, H->d_adj_frec_cells,
                                       H->d_adj_frec_order, (const T *)resid, H->n_adj_frec, H->nt_rec, n - 1, (T)1);
                }
                {
                    // step n-1 outside core2
                    dpmlk::AdjArgs<T> f = base(n - 1, 1 - acur);
                    f.lam = out1;
                    f.lam_o = lam;
                    f.lam_w = out2;
                    frame(f, H->d_adj_frame_s[0], H->n_adj_frame_s[0], core2, core2, H->side);
                }
                if (waves2 > 0) {
                    dpmlk::AdjArgs<T> c = base(n, acur);
                    c.lam = lam;
                    c.lam_o = lam_o;
                    c.lam_w = out1;
                    dpmlk::Adj2<T> q2{};
                    q2.un2 = (const T *)(hist + (size_t)(n - 1 - t0) * A.level);
                    q2.out1 = out1;
                    q2.out2 = out2;
                    for (int k = 0; k < 4; ++k) q2.s1[k] = core2s[k];
                    q2.t = -1;
                    if (H->nr > 0 && n - 1 < H->nt_rec) {
                        q2.rmap = H->d_rmap;
                        q2.rpool = H->d_rpool;
                        q2.resid = (const T *)resid;
                        q2.nt = H->nt_rec;
                        q2.t = n - 1;
                    }
                    hipLaunchKernelGGL((dpmlk::k_adjoint2_march2d<T, kAdjRows>), dim3((unsigned)round8((waves2 + 3) / 4)),
                                       ablock, 0, H->stream, c, q2, core2[0], core2[1], core2[2], core2[3], tiles2_x,
                                       waves2);
                }
                HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
                HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
                gather(out1, n - 1, H->stream);
                HIP_TRY(H, hipGetLastError());
                il = fr[1];          // a^{n-1}
                io = fr[0];          // a^n
                n -= 2;
                continue;
            }
            dpmlk::AdjArgs<T> q = base(n, acur);
            q.lam = lam;
            q.lam_o = lam_o;
            q.lam_w = lam_o;         // a^n over a^{n+2}
            if (march2d) {
                // the frame's cells on the side stream while the core marches on the
                // handle's stream (disjoint cells; joined before the next level)
                const bool fork = H->n_adj_frame > 0 && adj_waves > 0;
                if (fork) {
                    HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
                    HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
                }
                gather(lam, n, fork ? H->side : H->stream);
                frame(q, H->d_adj_frame, H->n_adj_frame, core, none, fork ? H->side : H->stream);
                if (adj_waves > 0)
                    hipLaunchKernelGGL((dpmlk::k_adjoint_march2d<T, kAdjRows>), mgrid, ablock, 0, H->stream, q,
                                       core[0], core[1], core[2], core[3], adj_tiles_x, adj_waves);
                if (fork) {
                    HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
                    HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
                }
            } else {
                gather(lam, n, H->stream);
                if (L.ndim == 2)
                    hipLaunchKernelGGL((dpmlk::k_adjoint_cell<T, 2>), agrid, ablock, 0, H->stream, q);
                else
                    hipLaunchKernelGGL((dpmlk::k_adjoint_cell<T, 3>), agrid, ablock, 0, H->stream, q);
            }
            HIP_TRY(H, hipGetLastError());
            std::swap(il, io);
            acur = 1 - acur;
            --n;
        }
        HIP_TRY(H, hipEventRecord(H->adj_sweep_done[seg & 1], H->stream));
    }
    // start: lam[io] holds a^1, slot 0 of segment 0's history U^0
    const T half_dt2 = (T)(0.5 * H->dt * H->dt);
    const T inv_h2 = (T)(1.0 / (H->h * H->h));
    if (L.ndim == 2)
        hipLaunchKernelGGL((dpmlk::k_adjoint_start<T, 2>), grid, block, 0, H->stream,
                           (const T *)(ws + A.off_lam[io]), (const T *)(ws + A.off_hist[0]), grad, half_dt2,
                           inv_h2, (int)L.N[0], (int)L.N[1], (int)L.N[2], (int)L.batch, (int64_t)L.ncell);
    else
        hipLaunchKernelGGL((dpmlk::k_adjoint_start<T, 3>), grid, block, 0, H->stream,
                           (const T *)(ws + A.off_lam[io]), (const T *)(ws + A.off_hist[0]), grad, half_dt2,
                           inv_h2, (int)L.N[0], (int)L.N[1], (int)L.N[2], (int)L.batch, (int64_t)L.ncell);
    HIP_TRY(H, hipGetLastError());
    H->recording = true;
    H->state_set = false;     // the fields now hold a recomputed intermediate level
    H->u_now = H->at(L.off_u[0]);     // and never point into the caller's workspace
    H->u_old = H->at(L.off_u[1]);
    H->cur = 0;
    return DPML_OK;
}

}  // namespace

extern "C" {

size_t dpml_adjoint_workspace_bytes(const dpml_t *H, int64_t nsteps, int64_t ckpt_every)
{
    if (!H || nsteps < 1 || ckpt_every < 1) return 0;
    return adj_layout(H, nsteps, ckpt_every).total;
}

int dpml_forward_checkpointed(dpml_t *H, int64_t nsteps, int64_t ckpt_every, void *adj_ws, size_t bytes)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 1 || ckpt_every < 1 || !adj_ws) return H->fail(DPML_EINVAL, "bad checkpoint arguments");
    if (!H->state_set || H->n != 0) return H->fail(DPML_ESTATE, "the forward run must start at time index 0");
    if (H->L.wall[0] || H->L.wall[1] || H->L.wall[2]) return H->fail(DPML_EINVAL, "the adjoint supports periodic grids only");
    if (bytes < adj_layout(H, nsteps, ckpt_every).total) return H->fail(DPML_ENOMEM, "adjoint workspace too small");
    if (((uintptr_t)adj_ws) % kAlign != 0) return H->fail(DPML_ENOMEM, "adjoint workspace must be 256-byte aligned");
    H->adj_ws = (char *)adj_ws;
    H->adj_bytes = bytes;
    H->adj_nsteps = nsteps;
    H->adj_every = ckpt_every;
    H->adj_ready = false;
    int rc = H->L.dtype == DPML_F32 ? forward_ckpt_impl<float>(H, nsteps) : forward_ckpt_impl<double>(H, nsteps);
    if (rc) return rc;
    H->adj_ready = true;
    return DPML_OK;
}

int dpml_adjoint(dpml_t *H, const void *resid, double *grad_c2, void *grad_w)
{
    if (!H) return DPML_EINVAL;
    if (!H->adj_ready) return H->fail(DPML_ESTATE, "no checkpointed forward run to differentiate");
    if (!grad_c2 || (H->nr > 0 && !resid)) return H->fail(DPML_EINVAL, "bad adjoint arguments");
    return H->L.dtype == DPML_F32 ? adjoint_impl<float>(H, resid, grad_c2, grad_w)
                                  : adjoint_impl<double>(H, resid, grad_c2, grad_w);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Many independent 2D problems of different sizes stepped by one launch per
// step (a flat tile work list over all problems), optionally captured with
// the whole step sequence into one HIP graph.
// ---------------------------------------------------------------------------
struct dpml_multi {
    int64_t count = 0;
    int dtype = 0;
    size_t esize = 4;
    std::vector<Layout> L;
    std::vector<double> h, dt;
    std::vector<size_t> base;        // workspace offset of each problem's block
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;       // private stream used only for graph capture
    size_t off_tiles = 0;            // single-step tile list (workspace)
    int64_t ntiles = 0;
    int vx = 1;
    int variant = DPML_VARIANT_MARCH;  // MARCH: single steps; TWOSTEP .. DEEP: multi-step passes
    int depth = 1;                   // levels per multi-step pass
    int tile_rows = 32;              // single steps: rows per marching tile
    int group = 4;                   // single steps: rows whose loads are issued together
    int pass_rows = 8;               // multi-step passes: rows per core wave
    int pass_group = 2;              // multi-step passes: rows whose loads are issued together
    // rotation state: U buffers holding levels n and n-1, aux buffer of level n
    int now = 0, old = 1, cur = 0;
    int64_t n = 0;
    bool state_set = false;
    // library-owned tables: step arguments per rotation state and role, and
    // the work lists of the multi-step passes ([levels - 2])
    std::vector<void *> d_args;      // [state * kRoles + role]
    dpmlk::TileRef *d_core_waves[kMaxLevels - 1] = {};
    int64_t n_core_waves[kMaxLevels - 1] = {-1, -1, -1, -1, -1, -1, -1};   // -1: not built for pass_rows yet
    dpmlk::Span2 *d_frame[kMaxLevels - 1][kMaxLevels] = {};
    int64_t n_frame[kMaxLevels - 1][kMaxLevels] = {};
    int pass_ok[kMaxLevels - 1] = {-1, -1, -1, -1, -1, -1, -1};   // every problem has a core (-1: not checked)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t graph_steps = -1;
    int graph_state = -1;
    std::string err;
    int fail(int code, const std::string &m) { err = m; return code; }
};

namespace {

thread_local std::string g_multi_error;

struct MultiLayout {
    std::vector<Layout> L;
    std::vector<size_t> base;
    size_t off_tiles = 0, total = 0;
    int64_t ntiles = 0;
    int vx = 1;
};

// The single-step tile list is sized for the shortest tiles allowed
// (kMultiMinRows rows); the default tiles are 256 VX columns x 32 rows,
// marched 4 rows at a time.  Each problem holds 2 + kMaxLevels U buffers (a
// pass of L levels writes U^{n+1} .. U^{n+L} while other waves still read
// U^n and U^{n-1}).
constexpr int kMultiMinRows = 4;
constexpr int kMultiTileRows = 32;
constexpr int kMultiGroup = 4;
constexpr int kMultiPassRows = 8;
constexpr int kMultiPassGroup = 2;
constexpr int kMultiUbufs = 2 + kMaxLevels;

// roles of the argument tables of one rotation state: a single step (role
// 0); then for passes of 2 .. kMaxLevels levels, in that order, the core
// and the pass's frame steps (levels + 1 roles each)
constexpr int kRoleStep = 0;
constexpr int kRoles = 1 + (kMaxLevels + 4) * (kMaxLevels - 1) / 2;

int role_base(int levels)
{
    int b = 1;
    for (int l = 2; l < levels; ++l) b += l + 1;
    return levels == 1 ? kRoleStep : b;
}

int state_key(int now, int old, int cur) { return (now * kMultiUbufs + old) * 2 + cur; }

std::string multi_layout(int64_t count, const dpml_grid_t *grids, MultiLayout &M)
{
    if (count < 1 || count > (1 << 20) || !grids) return "bad problem count";
    const int dtype = grids[0].dtype;
    size_t off = 0;
    bool even = true;
    M.L.resize((size_t)count);
    M.base.resize((size_t)count);
    for (int64_t p = 0; p < count; ++p) {
        if (grids[p].ndim != 2) return "multi-problem stepping is 2D only";
        if (grids[p].dtype != dtype) return "all problems must share one dtype";
        if (grids[p].batch > 1) return "multi-problem grids take no batch";
        if (grids[p].walls[0] || grids[p].walls[1]) return "multi-problem grids are periodic";
        std::string e = make_layout(&grids[p], false, M.L[p], kMultiUbufs);
        if (!e.empty()) return "problem " + std::to_string(p) + ": " + e;
        M.base[p] = off;
        off += align_up(M.L[p].total);
        even &= M.L[p].N[0] % 2 == 0;
    }
    M.vx = (dtype == DPML_F32 && even) ? 2 : 1;
    int64_t nt = 0;
    for (int64_t p = 0; p < count; ++p) {
        const int64_t tx = (M.L[p].N[0] + 256 * M.vx - 1) / (256 * M.vx);
        const int64_t ty = (M.L[p].N[1] + kMultiMinRows - 1) / kMultiMinRows;
        nt += tx * ty;
    }
    M.ntiles = nt;
    M.off_tiles = off; off += align_up((size_t)nt * sizeof(dpmlk::TileRef));
    M.total = off;
    return "";
}

// A throw-away single-problem view of problem p with U buffers `now` and
// `old` and aux buffer `cur` holding level n, so the single-problem argument
// builders can be reused.
dpml problem_view(const dpml_multi *H, int64_t p, int now, int old, int cur)
{
    dpml v;
    v.L = H->L[p];
    v.ws = H->ws + H->base[p];
    v.h = H->h[p];
    v.dt = H->dt[p];
    v.c2_const = 1.0;
    v.c2_field = false;
    v.cur = cur;
    v.u_now = v.at(v.L.off_u[now]);
    v.u_old = v.at(v.L.off_u[old]);
    return v;
}

// The kMaxLevels spare U buffers of a rotation state, in ascending order.
void spares(int now, int old, int s[kMaxLevels])
{
    int k = 0;
    for (int i = 0; i < kMultiUbufs && k < kMaxLevels; ++i)
        if (i != now && i != old) s[k++] = i;
}

template <typename T>
int multi_shape(dpml_multi *H);

template <typename T>
int multi_tables(dpml_multi *H, const double *const *sigmas)
{
    // damping tables of every problem
    for (int64_t p = 0; p < H->count; ++p) {
        dpml v = problem_view(H, p, 0, 1, 0);
        const double *sg[3] = {sigmas[3 * p], sigmas[3 * p + 1], nullptr};
        double one = 1.0;
        int rc = upload_tables<T>(&v, &one, 1, sg);
        if (rc) return H->fail(rc, v.err);
    }
    return multi_shape<T>(H);
}

// The single-step tile list for the handle's tile height (workspace); the
// argument tables built for earlier shapes are dropped.
template <typename T>
int multi_shape(dpml_multi *H)
{
    for (void *&d : H->d_args)
        if (d) { (void)hipFree(d); d = nullptr; }
    std::vector<dpmlk::TileRef> tiles;
    tiles.reserve((size_t)H->ntiles);
    for (int64_t p = 0; p < H->count; ++p) {
        const Layout &L = H->L[p];
        const int cw = 256 * H->vx;
        const int tx = (int)((L.N[0] + cw - 1) / cw);
        const int ty = (int)((L.N[1] + H->tile_rows - 1) / H->tile_rows);
        // cells [lo+1, lo+n) of an axis with a layer meet no damping term
        auto free_range = [&](int a, int64_t i0, int64_t i1) {
            return L.M[a] == 0 || (i0 >= L.lo[a] + 1 && i1 <= L.lo[a] + L.n[a]);
        };
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) {
                const int64_t x1 = std::min<int64_t>((int64_t)(x + 1) * cw, L.N[0]);
                const int64_t y1 = std::min<int64_t>((int64_t)(y + 1) * H->tile_rows, L.N[1]);
                const bool layer = !(free_range(0, (int64_t)x * cw, x1) && free_range(1, (int64_t)y * H->tile_rows, y1));
                tiles.push_back({(int32_t)p, x, y, layer ? 1 : 0});
            }
    }
    HIP_TRY(nullptr, hipMemcpy(H->ws + H->off_tiles, tiles.data(), tiles.size() * sizeof(tiles[0]),
                               hipMemcpyHostToDevice));
    H->ntiles = (int64_t)tiles.size();
    return DPML_OK;
}

// Upload a table into an empty slot (a filled slot may be read by work in
// flight and is never rewritten; the tables are dropped only after a sync).
template <typename T>
int upload_table(dpml_multi *H, int slot, const void *data, size_t bytes)
{
    if ((size_t)slot >= H->d_args.size()) H->d_args.resize((size_t)slot + 1, nullptr);
    if (H->d_args[slot]) return DPML_OK;
    HIP_TRY(nullptr, hipMalloc(&H->d_args[slot], bytes));
    HIP_TRY(nullptr, hipMemcpy(H->d_args[slot], data, bytes, hipMemcpyHostToDevice));
    return DPML_OK;
}

// Argument tables of rotation state (now, old, cur) for a pass of `levels`
// levels (1: one step in place; 2 .. 4: the core descriptors and the frame's
// steps, frame step j over everything outside the core shrunk by levels - j).
// Built once per state and depth (outside any capture) and kept.
template <typename T>
int ensure_state(dpml_multi *H, int now, int old, int cur, int levels)
{
    const int key = state_key(now, old, cur), rb = role_base(levels);
    const int nroles = levels == 1 ? 1 : levels + 1;
    bool have = true;
    for (int role = rb; role < rb + nroles; ++role) {
        const size_t slot = (size_t)key * kRoles + role;
        if (slot >= H->d_args.size() || !H->d_args[slot]) have = false;
    }
    if (have) return DPML_OK;
    const size_t c = (size_t)H->count;
    if (levels == 1) {
        std::vector<dpmlk::StepArgs<T>> step(c);
        for (int64_t p = 0; p < H->count; ++p) {
            dpml v = problem_view(H, p, now, old, cur);
            step[p] = make_args<T>(&v);
            step[p].tile_rows = H->tile_rows;
            step[p].tiles_x = (int)((v.L.N[0] + 256 * H->vx - 1) / (256 * H->vx));
        }
        return upload_table<T>(H, key * kRoles + kRoleStep, step.data(), c * sizeof(step[0]));
    }
    std::vector<dpmlk::MultiCore<T>> core(c);
    std::vector<std::vector<dpmlk::StepArgs<T>>> fr((size_t)levels, std::vector<dpmlk::StepArgs<T>>(c));
    int sp[kMaxLevels];
    spares(now, old, sp);
    // levels: U^n = now, U^{n-1} = old, U^{n+j} = spare j-1
    auto level_buf = [&](int j) { return j == 0 ? now : (j == -1 ? old : sp[j - 1]); };
    for (int64_t p = 0; p < H->count; ++p) {
        dpml v = problem_view(H, p, now, old, cur);
        int r[4];
        core_rect(v.L, levels, r);
        core[p].p = make_args<T>(&v);
        core[p].p.uout = (T *)v.at(v.L.off_u[sp[0]]);
        core[p].p.tile_rows = H->pass_rows;
        for (int k = 0; k < 4; ++k) core[p].p.skip[k] = r[k];
        core[p].next2 = (T *)v.at(v.L.off_u[sp[1]]);
        core[p].next3 = levels == 3 ? (T *)v.at(v.L.off_u[sp[2]]) : nullptr;
        core[p].pen = (T *)v.at(v.L.off_u[sp[levels - 2]]);
        core[p].fin = (T *)v.at(v.L.off_u[sp[levels - 1]]);
        for (int j = 1; j <= levels; ++j) {
            const int sh = levels - j;
            dpml w = problem_view(H, p, level_buf(j - 1), level_buf(j - 2), (j % 2 == 0) ? 1 - cur : cur);
            fr[j - 1][p] = make_args<T>(&w);
            fr[j - 1][p].uout = (T *)w.at(w.L.off_u[sp[j - 1]]);
            fr[j - 1][p].skip[0] = r[0] + sh;
            fr[j - 1][p].skip[1] = r[1] - sh;
            fr[j - 1][p].skip[2] = r[2] + sh;
            fr[j - 1][p].skip[3] = r[3] - sh;
        }
    }
    int rc = upload_table<T>(H, key * kRoles + rb, core.data(), c * sizeof(core[0]));
    for (int j = 1; j <= levels && !rc; ++j)
        rc = upload_table<T>(H, key * kRoles + rb + j, fr[j - 1].data(), c * sizeof(fr[j - 1][0]));
    return rc;
}

// Do all problems have a core for passes of `levels` levels?
bool multi_pass_ok(dpml_multi *H, int levels)
{
    int &ok = H->pass_ok[levels - 2];
    if (ok < 0) {
        ok = 1;
        for (int64_t p = 0; p < H->count; ++p) {
            int r[4];
            core_rect(H->L[p], levels, r);
            if (H->L[p].N[0] < 8 || H->L[p].N[1] < 8 || r[1] - r[0] < 1 || r[3] - r[2] < 1) ok = 0;
        }
    }
    return ok == 1;
}

// Work lists of the passes of `levels` levels: the core waves (problem,
// strip, tile row) for pass_rows, and for frame step j the spans outside
// each core shrunk by levels - j.
int ensure_pass_lists(dpml_multi *H, int levels)
{
    const int q = levels - 2;
    if (H->n_core_waves[q] >= 0) return DPML_OK;
    std::vector<dpmlk::TileRef> waves;
    std::vector<dpmlk::Span2> fr[kMaxLevels];
    for (int64_t p = 0; p < H->count; ++p) {
        const Layout &L = H->L[p];
        int r[4];
        core_rect(L, levels, r);
        const int VX = multistep_vx(L);
        const int HL = (levels + VX - 1) / VX;
        const int sw = (64 - 2 * HL) * VX;
        const int strips = (r[1] - r[0] + sw - 1) / sw;
        const int tys = (r[3] - r[2] + H->pass_rows - 1) / H->pass_rows;
        for (int ty = 0; ty < tys; ++ty)
            for (int s = 0; s < strips; ++s) waves.push_back({(int32_t)p, s, ty, 0});
        for (int j = 1; j <= levels; ++j) {
            const int sh = levels - j;
            const int S[4] = {r[0] + sh, r[1] - sh, r[2] + sh, r[3] - sh};
            frame_spans(L, S, (int)p, fr[j - 1]);
        }
    }
    HIP_TRY(nullptr, hipMalloc((void **)&H->d_core_waves[q], std::max<size_t>(1, waves.size()) * sizeof(waves[0])));
    HIP_TRY(nullptr, hipMemcpy(H->d_core_waves[q], waves.data(), waves.size() * sizeof(waves[0]),
                               hipMemcpyHostToDevice));
    for (int j = 0; j < levels; ++j) {
        HIP_TRY(nullptr, hipMalloc((void **)&H->d_frame[q][j], std::max<size_t>(1, fr[j].size()) * sizeof(fr[j][0])));
        HIP_TRY(nullptr, hipMemcpy(H->d_frame[q][j], fr[j].data(), fr[j].size() * sizeof(fr[j][0]),
                                   hipMemcpyHostToDevice));
        H->n_frame[q][j] = (int64_t)fr[j].size();
    }
    H->n_core_waves[q] = (int64_t)waves.size();
    if (!H->side) HIP_TRY(nullptr, hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking));
    if (!H->ev_fork) HIP_TRY(nullptr, hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
    if (!H->ev_join) HIP_TRY(nullptr, hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
    return DPML_OK;
}

// Drop the work lists (after a change of pass_rows).
void drop_pass_lists(dpml_multi *H)
{
    for (int q = 0; q < kMaxLevels - 1; ++q) {
        if (H->d_core_waves[q]) { (void)hipFree(H->d_core_waves[q]); H->d_core_waves[q] = nullptr; }
        for (int j = 0; j < kMaxLevels; ++j)
            if (H->d_frame[q][j]) { (void)hipFree(H->d_frame[q][j]); H->d_frame[q][j] = nullptr; }
        H->n_core_waves[q] = -1;
    }
}

template <typename T>
int multi_launch_step(dpml_multi *H, hipStream_t s, int key)
{
    const dim3 grid((unsigned)round8((int)H->ntiles)), block(256);
    const auto *probs = (const dpmlk::StepArgs<T> *)H->d_args[(size_t)key * kRoles + kRoleStep];
    const auto *tiles = (const dpmlk::TileRef *)(H->ws + H->off_tiles);
    constexpr int V2 = sizeof(T) == 4 ? 2 : 1;
#define DPML_MULTI2D(VX_, R_) \
    hipLaunchKernelGGL((dpmlk::k_step_multi2d<T, VX_, R_>), grid, block, 0, s, probs, tiles, (int)H->ntiles)
    if (H->vx == 2) {
        if (H->group == 4) DPML_MULTI2D(V2, 4);
        else if (H->group == 2) DPML_MULTI2D(V2, 2);
        else DPML_MULTI2D(V2, 1);
    } else {
        if (H->group == 4) DPML_MULTI2D(1, 4);
        else if (H->group == 2) DPML_MULTI2D(1, 2);
        else DPML_MULTI2D(1, 1);
    }
#undef DPML_MULTI2D
    HIP_TRY(nullptr, hipGetLastError());
    return DPML_OK;
}

// One pass of `levels` levels over every problem: the core waves on stream
// s, the frame's steps on the side stream meanwhile (fork/join events).
template <typename T>
int multi_launch_pass(dpml_multi *H, hipStream_t s, int key, int levels)
{
    constexpr int VX = sizeof(T) == 4 ? 4 : 2;
    const int q = levels - 2, rb = role_base(levels);
    const auto *cores = (const dpmlk::MultiCore<T> *)H->d_args[(size_t)key * kRoles + rb];
    const dim3 block(256);
    HIP_TRY(nullptr, hipEventRecord(H->ev_fork, s));
    HIP_TRY(nullptr, hipStreamWaitEvent(H->side, H->ev_fork, 0));
    const int nw = (int)H->n_core_waves[q];
    const dim3 grid((unsigned)round8((nw + 3) / 4));
    const dpmlk::TileRef *wl = H->d_core_waves[q];
#define DPML_MULTI_PASS(KER)                                                                          \
    if (H->pass_group == 4) hipLaunchKernelGGL((dpmlk::KER<T, VX, 4>), grid, block, 0, s, cores, wl, nw); \
    else if (H->pass_group == 1) hipLaunchKernelGGL((dpmlk::KER<T, VX, 1>), grid, block, 0, s, cores, wl, nw); \
    else hipLaunchKernelGGL((dpmlk::KER<T, VX, 2>), grid, block, 0, s, cores, wl, nw);
#define DPML_MULTI_PASS_N(NL)                                                                               \
    if (H->pass_group == 4) hipLaunchKernelGGL((dpmlk::k_multi_stepN_march<T, VX, 4, NL>), grid, block, 0, s, cores, wl, nw); \
    else if (H->pass_group == 1) hipLaunchKernelGGL((dpmlk::k_multi_stepN_march<T, VX, 1, NL>), grid, block, 0, s, cores, wl, nw); \
    else hipLaunchKernelGGL((dpmlk::k_multi_stepN_march<T, VX, 2, NL>), grid, block, 0, s, cores, wl, nw);
    switch (levels) {
    case 2: { DPML_MULTI_PASS(k_multi_step2_march) } break;
    case 3: { DPML_MULTI_PASS(k_multi_step3_march) } break;
    case 4: { DPML_MULTI_PASS_N(4) } break;
    case 5: { DPML_MULTI_PASS_N(5) } break;
    case 6: { DPML_MULTI_PASS_N(6) } break;
    case 7: { DPML_MULTI_PASS_N(7) } break;
    default: { DPML_MULTI_PASS_N(8) } break;
    }
#undef DPML_MULTI_PASS
#undef DPML_MULTI_PASS_N
    for (int j = 1; j <= levels; ++j) {
        const int nf = (int)H->n_frame[q][j - 1];
        const auto *fa = (const dpmlk::StepArgs<T> *)H->d_args[(size_t)key * kRoles + rb + j];
        if (nf > 0)
            hipLaunchKernelGGL((dpmlk::k_multi_frame_march<T, kFrameGroup>), dim3((unsigned)round8((nf + 3) / 4)),
                               block, 0, H->side, fa, H->d_frame[q][j - 1], nf);
    }
    HIP_TRY(nullptr, hipEventRecord(H->ev_join, H->side));
    HIP_TRY(nullptr, hipStreamWaitEvent(s, H->ev_join, 0));
    HIP_TRY(nullptr, hipGetLastError());
    return DPML_OK;
}

// nsteps steps from the handle's rotation state: passes of the variant's
// depth (2 .. kMaxLevels levels), shorter ones for the last steps or where
// a problem has no core that deep, and single steps where none has.  kPrepare only
// builds the tables the run needs (before a capture); kLaunch enqueues the
// run on stream s and advances the rotation state; kAdvance only advances
// it (after a graph replay).
enum { kPrepare = 0, kLaunch = 1, kAdvance = 2 };

template <typename T>
int multi_run(dpml_multi *H, hipStream_t s, int64_t nsteps, int mode)
{
    const int want = H->variant == DPML_VARIANT_MARCH ? 1 : H->depth;
    int now = H->now, old = H->old, cur = H->cur;
    int64_t k = 0;
    while (k < nsteps) {
        int lv = (int)std::min<int64_t>(want, nsteps - k);
        while (lv >= 2 && !multi_pass_ok(H, lv)) --lv;
        int rc = DPML_OK;
        if (mode != kAdvance) {
            if (lv >= 2) rc = ensure_pass_lists(H, lv);
            if (!rc) rc = ensure_state<T>(H, now, old, cur, lv);
        }
        if (!rc && mode == kLaunch)
            rc = lv == 1 ? multi_launch_step<T>(H, s, state_key(now, old, cur))
                         : multi_launch_pass<T>(H, s, state_key(now, old, cur), lv);
        if (rc) return rc;
        if (lv == 1) {
            std::swap(now, old);
        } else {
            int sp[kMaxLevels];
            spares(now, old, sp);
            now = sp[lv - 1];
            old = sp[lv - 2];
        }
        if (lv % 2) cur = 1 - cur;
        k += lv;
    }
    if (mode != kPrepare) {
        H->now = now;
        H->old = old;
        H->cur = cur;
        H->n += nsteps;
    }
    return DPML_OK;
}

template <typename T>
int multi_step_impl(dpml_multi *H, int64_t nsteps, bool use_graph)
{
    if (!use_graph) {
        int rc = multi_run<T>(H, H->stream, nsteps, kLaunch);
        return rc ? H->fail(rc, g_create_error) : DPML_OK;
    }
    const int state = state_key(H->now, H->old, H->cur);
    if (!(H->exec && H->graph_steps == nsteps && H->graph_state == state)) {
        if (H->exec) {
            // the replaced graph may still run on the stream: wait before its release
            hipError_t es = hipStreamSynchronize(H->stream);
            if (es != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(es));
            (void)hipGraphExecDestroy(H->exec);
            H->exec = nullptr;
        }
        if (H->graph) { (void)hipGraphDestroy(H->graph); H->graph = nullptr; }
        if (!H->cap) {
            hipError_t e = hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking);
            if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
        }
        int rc = multi_run<T>(H, H->cap, nsteps, kPrepare);     // tables before the capture
        if (rc) return H->fail(rc, g_create_error);
        const int now = H->now, old = H->old, cur = H->cur;
        const int64_t n0 = H->n;
        hipError_t e = hipStreamBeginCapture(H->cap, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
        rc = multi_run<T>(H, H->cap, nsteps, kLaunch);
        e = hipStreamEndCapture(H->cap, &H->graph);
        // the capture only recorded the launches: the state advances at the replay
        H->now = now;
        H->old = old;
        H->cur = cur;
        H->n = n0;
        if (rc) return H->fail(rc, g_create_error);
        if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
        e = hipGraphInstantiate(&H->exec, H->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
        H->graph_steps = nsteps;
        H->graph_state = state;
    }
    hipError_t e = hipGraphLaunch(H->exec, H->stream);
    if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
    return multi_run<T>(H, H->stream, nsteps, kAdvance);
}

}  // namespace
extern "C" {

size_t dpml_multi_workspace_bytes(int64_t count, const dpml_grid_t *grids)
{
    MultiLayout M;
    if (!multi_layout(count, grids, M).empty()) return 0;
    return M.total;
}

int dpml_multi_create(int64_t count, const dpml_grid_t *grids, const double *h, const double *dt,
                      const double *const *sigmas, void *workspace, size_t ws_bytes, void *stream,
                      dpml_multi_t **out)
{
    if (!out) { g_multi_error = "out is NULL"; return DPML_EINVAL; }
    *out = nullptr;
    MultiLayout M;
    std::string e = multi_layout(count, grids, M);
    if (!e.empty()) { g_multi_error = e; return DPML_EINVAL; }
    if (!h || !dt || !sigmas) { g_multi_error = "h, dt and sigmas are required"; return DPML_EINVAL; }
    for (int64_t p = 0; p < count; ++p) {
        const Layout &L = M.L[p];
        if (!(h[p] > 0) || !(dt[p] > 0) || !std::isfinite(h[p]) || !std::isfinite(dt[p])) {
            g_multi_error = "problem " + std::to_string(p) + ": h and dt must be positive"; return DPML_EINVAL;
        }
        if (dt[p] / h[p] * std::sqrt(2.0) > 1.0) {
            g_multi_error = "problem " + std::to_string(p) + ": time step violates dt/h sqrt(2) <= 1"; return DPML_EINVAL;
        }
        for (int a = 0; a < 2; ++a) {
            const double *sg = sigmas[3 * p + a];
            if (!sg) continue;
            for (int64_t i = 0; i < L.N[a]; ++i) {
                if (!(sg[i] >= 0) || !std::isfinite(sg[i]) || dt[p] * sg[i] > 4.0 ||
                    (sg[i] != 0 && i >= L.lo[a] && i < L.lo[a] + L.n[a])) {
                    g_multi_error = "problem " + std::to_string(p) + ": invalid sigma"; return DPML_EINVAL;
                }
            }
        }
    }
    if (!workspace || ws_bytes < M.total) { g_multi_error = "workspace too small"; return DPML_ENOMEM; }
    if (((uintptr_t)workspace) % kAlign != 0) { g_multi_error = "workspace must be 256-byte aligned"; return DPML_ENOMEM; }
    dpml_multi *H = new (std::nothrow) dpml_multi();
    if (!H) { g_multi_error = "out of host memory"; return DPML_ENOMEM; }
    H->count = count;
    H->dtype = grids[0].dtype;
    H->esize = H->dtype == DPML_F32 ? 4 : 8;
    H->L = M.L;
    H->base = M.base;
    H->h.assign(h, h + count);
    H->dt.assign(dt, dt + count);
    H->ws = (char *)workspace;
    H->stream = (hipStream_t)stream;
    H->off_tiles = M.off_tiles;
    H->ntiles = M.ntiles;
    H->vx = M.vx;
    H->tile_rows = kMultiTileRows;
    H->group = kMultiGroup;
    H->pass_rows = kMultiPassRows;
    H->pass_group = kMultiPassGroup;
    int rc = H->dtype == DPML_F32 ? multi_tables<float>(H, sigmas) : multi_tables<double>(H, sigmas);
    if (rc) { g_multi_error = H->err.empty() ? g_create_error : H->err; delete H; return rc; }
    *out = H;
    return DPML_OK;
}

int dpml_multi_set_state(dpml_multi_t *H, const void *const *U0)
{
    if (!H) return DPML_EINVAL;
    if (!U0) return H->fail(DPML_EINVAL, "U0 is NULL");
    for (int64_t p = 0; p < H->count; ++p) {
        if (!U0[p]) return H->fail(DPML_EINVAL, "U0[" + std::to_string(p) + "] is NULL");
        dpml v = problem_view(H, p, 0, 1, 0);
        v.stream = H->stream;
        int rc = H->dtype == DPML_F32 ? set_state_impl<float>(&v, U0[p], nullptr)
                                      : set_state_impl<double>(&v, U0[p], nullptr);
        if (rc) return H->fail(rc, v.err);
    }
    H->now = 0;
    H->old = 1;
    H->cur = 0;
    H->n = 0;
    H->state_set = true;
    return DPML_OK;
}

int dpml_multi_step(dpml_multi_t *H, int64_t nsteps, int32_t use_graph)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0) return H->fail(DPML_EINVAL, "nsteps < 0");
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_multi_set_state has not been called");
    if (nsteps == 0) return DPML_OK;
    return H->dtype == DPML_F32 ? multi_step_impl<float>(H, nsteps, use_graph != 0)
                                : multi_step_impl<double>(H, nsteps, use_graph != 0);
}

int dpml_multi_field(dpml_multi_t *H, int64_t prob, int32_t which, void **ptr, int64_t shape[3])
{
    if (!H || !ptr || !shape || prob < 0 || prob >= H->count) return DPML_EINVAL;
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_multi_set_state has not been called");
    const Layout &L = H->L[prob];
    char *b = H->ws + H->base[prob];
    for (int a = 0; a < 3; ++a) shape[a] = L.N[a];
    const int q = H->cur;
    if (which == DPML_FIELD_U) { *ptr = b + L.off_u[H->now]; return DPML_OK; }
    if (which == DPML_FIELD_UPREV) { *ptr = b + L.off_u[H->old]; return DPML_OK; }
    const int a = (which - 2) / 2;
    if (which < 2 || a >= L.ndim || L.M[a] == 0) return H->fail(DPML_EINVAL, "no such field");
    shape[a] = L.M[a] + 1;
    *ptr = b + ((which % 2 == 0) ? L.off_phi[a][q] : L.off_psi[a][q]);
    return DPML_OK;
}

int64_t dpml_multi_tiles(const dpml_multi_t *H) { return H ? H->ntiles : -1; }

int dpml_multi_set_variant(dpml_multi_t *H, int32_t variant, int32_t tile_rows, int32_t group)
{
    if (!H) return DPML_EINVAL;
    if (variant == DPML_VARIANT_AUTO) variant = DPML_VARIANT_MARCH;
    if (variant != DPML_VARIANT_MARCH && variant != DPML_VARIANT_TWOSTEP && variant != DPML_VARIANT_THREESTEP &&
        variant != DPML_VARIANT_FOURSTEP && variant != DPML_VARIANT_DEEP)
        return H->fail(DPML_EINVAL, "variant must be DPML_VARIANT_MARCH, TWOSTEP, THREESTEP, FOURSTEP or DEEP");
    const bool pass = variant != DPML_VARIANT_MARCH;
    const int depth = pass_depth(variant, tile_rows);
    if (variant == DPML_VARIANT_DEEP) {
        if (tile_rows < 0 || tile_rows >= (1 << 24) || depth < 2 || depth > kMaxLevels)
            return H->fail(DPML_EINVAL, "DEEP passes take 2 .. 8 levels (tile_rows bits 20-23)");
        tile_rows &= 0xFFFFF;
    }
    if (tile_rows == 0) tile_rows = pass ? kMultiPassRows : kMultiTileRows;
    if (group == 0) group = pass ? kMultiPassGroup : kMultiGroup;
    if (tile_rows < (pass ? 1 : kMultiMinRows) || tile_rows > 4096 || (group != 1 && group != 2 && group != 4))
        return H->fail(DPML_EINVAL, "tile_rows must be in [4, 4096] ([1, 4096] for TWOSTEP) and group 1, 2 or 4");
    hipError_t e = hipStreamSynchronize(H->stream);       // the tables may be in use
    if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
    if (H->exec) { (void)hipGraphExecDestroy(H->exec); H->exec = nullptr; }
    if (H->graph) { (void)hipGraphDestroy(H->graph); H->graph = nullptr; }
    H->graph_steps = -1;
    H->variant = variant;
    H->depth = depth;
    if (pass) {
        if (tile_rows != H->pass_rows) drop_pass_lists(H);
        H->pass_rows = tile_rows;
        H->pass_group = group;
        for (void *&d : H->d_args)                      // the core tables hold the wave height
            if (d) { (void)hipFree(d); d = nullptr; }
        return DPML_OK;
    }
    H->tile_rows = tile_rows;
    H->group = group;
    int rc = H->dtype == DPML_F32 ? multi_shape<float>(H) : multi_shape<double>(H);
    return rc ? H->fail(rc, H->err.empty() ? g_create_error : H->err) : DPML_OK;
}

int dpml_multi_sync(dpml_multi_t *H)
{
    if (!H) return DPML_EINVAL;
    hipError_t e = hipStreamSynchronize(H->stream);
    if (e != hipSuccess) return H->fail(DPML_EHIP, hipGetErrorString(e));
    return DPML_OK;
}

void dpml_multi_destroy(dpml_multi_t *H)
{
    if (!H) return;
    (void)hipStreamSynchronize(H->stream);
    if (H->exec) (void)hipGraphExecDestroy(H->exec);
    if (H->graph) (void)hipGraphDestroy(H->graph);
    if (H->cap) (void)hipStreamDestroy(H->cap);
    for (void *d : H->d_args)
        if (d) (void)hipFree(d);
    drop_pass_lists(H);
    if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
    if (H->ev_join) (void)hipEventDestroy(H->ev_join);
    if (H->side) (void)hipStreamDestroy(H->side);
    delete H;
}

const char *dpml_multi_last_error(const dpml_multi_t *H) { return H ? H->err.c_str() : g_multi_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// RK4 (the paper's integrator) on the handle's grid
// ---------------------------------------------------------------------------
namespace {

struct RKLayout {
    size_t off_u[4], off_v[4], off_phi[4][3], off_psi[4][3], total;
};

RKLayout rk_layout(const Layout &L)
{
    RKLayout R{};
    size_t off = 0;
    const size_t ub = align_up((size_t)L.ncell * L.esize);
    for (int k = 0; k < 4; ++k) {
        R.off_u[k] = off; off += ub;
        R.off_v[k] = off; off += ub;
        for (int a = 0; a < L.ndim; ++a) {
            if (L.M[a] == 0) continue;
            const size_t ab = align_up((size_t)L.aux_elems[a] * L.esize);
            R.off_phi[k][a] = off; off += ab;
            R.off_psi[k][a] = off; off += ab;
        }
    }
    R.total = off;
    return R;
}

template <typename T>
dpmlk::RKFields<T> rk_fields(dpml *H, const RKLayout &R, int set)
{
    dpmlk::RKFields<T> f{};
    f.u = (T *)(H->rk_ws + R.off_u[set]);
    f.v = (T *)(H->rk_ws + R.off_v[set]);
    for (int a = 0; a < 3; ++a) {
        f.phi[a] = (a < H->L.ndim && H->L.M[a] > 0) ? (T *)(H->rk_ws + R.off_phi[set][a]) : nullptr;
        f.psi[a] = (a < H->L.ndim && H->L.M[a] > 0) ? (T *)(H->rk_ws + R.off_psi[set][a]) : nullptr;
    }
    return f;
}

template <typename T>
int rk4_step_impl(dpml *H, int64_t nsteps)
{
    const Layout &L = H->L;
    const RKLayout R = rk_layout(L);
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    const double wgt[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    dim3 block(64, 4, 1);
    dim3 grid((unsigned)((L.N[0] + 63) / 64), (unsigned)((L.N[1] + 3) / 4), (unsigned)(L.ndim == 3 ? L.N[2] : 1));
    for (int64_t k = 0; k < nsteps; ++k) {
        int *role = H->rk_role;   // role[0] = Y0, role[1] = YS0, role[2] = YS1, role[3] = S
        for (int st = 0; st < 4; ++st) {
            dpmlk::RKArgs<T> q{};
            for (int a = 0; a < 3; ++a) q.ax[a] = make_axis<T>(H, a, false);
            q.y0 = rk_fields<T>(H, R, role[0]);
            q.yin = st == 0 ? q.y0 : rk_fields<T>(H, R, role[1 + (st - 1) % 2]);
            q.yout = rk_fields<T>(H, R, role[1 + st % 2]);
            q.s = rk_fields<T>(H, R, role[3]);
            q.c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
            q.c2_const = (T)H->c2_const;
            q.inv_h2 = (T)(1.0 / (H->h * H->h));
            q.inv_h = (T)(1.0 / H->h);
            q.inv_2h = (T)(1.0 / (2.0 * H->h));
            q.w = (T)wgt[st];
            q.w3 = (T)wgt[3];
            q.cdt = st < 3 ? (T)(cst[st + 1] * H->dt) : T(0);
            q.dt = (T)H->dt;
            q.stage = st;
            q.nx = (int32_t)L.N[0];
            q.ny = (int32_t)L.N[1];
            q.nz = (int32_t)L.N[2];
            if (L.ndim == 2)
                hipLaunchKernelGGL((dpmlk::k_rk4_stage<T, 2>), grid, block, 0, H->stream, q);
            else
                hipLaunchKernelGGL((dpmlk::k_rk4_stage<T, 3>), grid, block, 0, H->stream, q);
            HIP_TRY(H, hipGetLastError());
        }
        std::swap(role[0], role[3]);   // S now holds y^{n+1}
        H->rk_n += 1;
    }
    return DPML_OK;
}

}  // namespace

extern "C" {

size_t dpml_rk4_workspace_bytes(const dpml_t *H)
{
    if (!H || H->L.batch != 1) return 0;
    return rk_layout(H->L).total;
}

int dpml_rk4_set_state(dpml_t *H, void *rk_ws, size_t bytes, const void *U0, const void *V0)
{
    if (!H) return DPML_EINVAL;
    if (H->L.batch != 1) return H->fail(DPML_EINVAL, "RK4 stepping takes no batch");
    if (H->L.wall[0] || H->L.wall[1] || H->L.wall[2]) return H->fail(DPML_EINVAL, "RK4 stepping supports periodic grids only");
    if (!rk_ws || !U0) return H->fail(DPML_EINVAL, "rk_ws and U0 are required");
    const RKLayout R = rk_layout(H->L);
    if (bytes < R.total) return H->fail(DPML_ENOMEM, "RK4 workspace too small");
    if (((uintptr_t)rk_ws) % kAlign != 0) return H->fail(DPML_ENOMEM, "RK4 workspace must be 256-byte aligned");
    H->rk_ws = (char *)rk_ws;
    for (int k = 0; k < 4; ++k) H->rk_role[k] = k;
    HIP_TRY(H, hipMemsetAsync(rk_ws, 0, R.total, H->stream));
    const size_t ub = (size_t)H->L.ncell * H->L.esize;
    HIP_TRY(H, hipMemcpyAsync(H->rk_ws + R.off_u[0], U0, ub, hipMemcpyDeviceToDevice, H->stream));
    if (V0) HIP_TRY(H, hipMemcpyAsync(H->rk_ws + R.off_v[0], V0, ub, hipMemcpyDeviceToDevice, H->stream));
    H->rk_n = 0;
    H->rk_set = true;
    return DPML_OK;
}

int dpml_rk4_step(dpml_t *H, int64_t nsteps)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0) return H->fail(DPML_EINVAL, "nsteps < 0");
    if (!H->rk_set) return H->fail(DPML_ESTATE, "dpml_rk4_set_state has not been called");
    return H->L.dtype == DPML_F32 ? rk4_step_impl<float>(H, nsteps) : rk4_step_impl<double>(H, nsteps);
}

int dpml_rk4_field(dpml_t *H, int32_t which, void **ptr, int64_t shape[3])
{
    if (!H || !ptr || !shape) return DPML_EINVAL;
    if (!H->rk_set) return H->fail(DPML_ESTATE, "dpml_rk4_set_state has not been called");
    const Layout &L = H->L;
    const RKLayout R = rk_layout(L);
    const int set = H->rk_role[0];
    for (int a = 0; a < 3; ++a) shape[a] = L.N[a];
    if (which == DPML_FIELD_U) { *ptr = H->rk_ws + R.off_u[set]; return DPML_OK; }
    if (which == 1) { *ptr = H->rk_ws + R.off_v[set]; return DPML_OK; }
    const int a = (which - 2) / 2;
    if (which < 2 || a >= L.ndim || L.M[a] == 0) return H->fail(DPML_EINVAL, "no such field");
    shape[a] = L.M[a] + 1;
    *ptr = H->rk_ws + ((which % 2 == 0) ? R.off_phi[set][a] : R.off_psi[set][a]);
    return DPML_OK;
}

int64_t dpml_rk4_time_index(const dpml_t *H) { return H && H->rk_set ? H->rk_n : -1; }

}  // extern "C"

// ---------------------------------------------------------------------------
// HIP-graph replay of a run of steps on the single-problem handle
// ---------------------------------------------------------------------------
namespace {

template <typename T>
int step_graph_impl(dpml *H, int64_t nsteps)
{
    const bool reuse = H->exec && H->graph_steps == nsteps && H->graph_cur == H->cur &&
                       H->graph_unow == H->u_now && H->graph_uold == H->u_old &&
                       H->graph_variant == H->variant && H->graph_rows == H->tile_rows;
    if (!reuse) {
        if (H->exec) {
            // the replaced graph may still run on the stream: wait before its release
            HIP_TRY(H, hipStreamSynchronize(H->stream));
            (void)hipGraphExecDestroy(H->exec);
            H->exec = nullptr;
        }
        if (H->graph) { (void)hipGraphDestroy(H->graph); H->graph = nullptr; }
        if (!H->cap) HIP_TRY(H, hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
        // capture on a private stream with a throw-away copy of the rotation state
        dpml view = *H;
        view.stream = H->cap;
        view.err.clear();
        view.timing = false;
        const int top = multistep_levels(H, nsteps);   // passes take at most this many levels
        for (int lv = 2; lv <= top; ++lv) {    // frame tables, side stream, events before capture
            int rcf = ensure_multistep(H, lv);
            if (rcf) return rcf;
            view.d_ffused[lv - 2] = H->d_ffused[lv - 2];
            view.n_ffused[lv - 2] = H->n_ffused[lv - 2];
            for (int sh = 0; sh < kMaxLevels; ++sh) {
                view.d_frame[lv - 2][sh] = H->d_frame[lv - 2][sh];
                view.n_frame[lv - 2][sh] = H->n_frame[lv - 2][sh];
                view.d_fspan[lv - 2][sh] = H->d_fspan[lv - 2][sh];
                view.n_fspan[lv - 2][sh] = H->n_fspan[lv - 2][sh];
                view.fspan_rows = H->fspan_rows;
            }
        }
        {
            int rcs = ensure_side(H);
            if (rcs) return rcs;
        }
        view.side = H->side;
        view.ev_fork = H->ev_fork;
        view.ev_join = H->ev_join;
        HIP_TRY(H, hipStreamBeginCapture(H->cap, hipStreamCaptureModeRelaxed));
        int rc = step_impl<T>(&view, nsteps);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(H->cap, &g);
        view.cap = nullptr; view.graph = nullptr; view.exec = nullptr;   // not owned by the view
        view.d_src_cells = view.d_src_order = view.d_rec_cells = view.d_rec_sorted = view.d_rec_order = nullptr;
        for (int lv = 0; lv < kMaxLevels - 1; ++lv) view.d_ffused[lv] = nullptr;
        for (int lv = 0; lv < kMaxLevels - 1; ++lv)
            for (int sh = 0; sh < kMaxLevels; ++sh) {
                view.d_frame[lv][sh] = nullptr;
                view.d_fspan[lv][sh] = nullptr;
            }
        view.side = nullptr;
        view.ev_fork = view.ev_join = nullptr;
        H->graph_end_unow = view.u_now;
        H->graph_end_uold = view.u_old;
        H->graph_end_cur = view.cur;
        if (rc) return H->fail(rc, view.err);
        if (e != hipSuccess) return hip_fail(H, e, "hipStreamEndCapture");
        H->graph = g;
        HIP_TRY(H, hipGraphInstantiate(&H->exec, H->graph, nullptr, nullptr, 0));
        H->graph_steps = nsteps;
        H->graph_cur = H->cur;
        H->graph_unow = H->u_now;
        H->graph_uold = H->u_old;
        H->graph_variant = H->variant;
        H->graph_rows = H->tile_rows;
    }
    HIP_TRY(H, hipGraphLaunch(H->exec, H->stream));
    H->u_now = H->graph_end_unow;
    H->u_old = H->graph_end_uold;
    H->cur = H->graph_end_cur;
    H->n += nsteps;
    return DPML_OK;
}

}  // namespace

extern "C" int dpml_step_graph(dpml_t *H, int64_t nsteps)
{
    if (!H) return DPML_EINVAL;
    if (nsteps < 0) return H->fail(DPML_EINVAL, "nsteps < 0");
    if (!H->state_set) return H->fail(DPML_ESTATE, "dpml_set_state has not been called");
    if (H->ns > 0 || H->nr > 0 || H->plane_axis >= 0)
        return H->fail(DPML_EINVAL, "graph replay needs a run without sources, receivers or planes");
    if (nsteps == 0) return DPML_OK;
    return H->L.dtype == DPML_F32 ? step_graph_impl<float>(H, nsteps) : step_graph_impl<double>(H, nsteps);
}
