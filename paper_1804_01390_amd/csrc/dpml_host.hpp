// dpml_host.hpp -- internal to the library: the workspace layout, the handle
// struct and the small host helpers shared by the translation units of
// libdpml.so (dpml.hip: the C ABI, 2D paths, adjoint, RK4, problem sets;
// dpml3d.hip: the 3D stepping paths).  Not installed, not part of the ABI.
#pragma once

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
#include <vector>

namespace dpmlh {

inline thread_local std::string g_create_error;



inline constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int ndim = 0;
    int dtype = 0;
    size_t esize = 0;
    int64_t N[3] = {1, 1, 1};
    int64_t n[3] = {1, 1, 1};
    int32_t lo[3] = {0, 0, 0};
    int32_t hi[3] = {0, 0, 0};
    int32_t M[3] = {0, 0, 0};
    int32_t wall[3] = {0, 0, 0};        // reflecting walls instead of periodic wrap
    int64_t ncell = 0;                  // cells of one problem
    int64_t batch = 1;                  // independent problems sharing c^2 and sigma
    int64_t aux_elems[3] = {0, 0, 0};   // elements of one compact aux array (one problem)
    // byte offsets into the workspace
    int n_ubuf = 2;                     // U buffers: U^n, U^{n-1} (+ spares of the multi-step variants)
    size_t off_u[10] = {};
    size_t off_c2 = 0;
    size_t off_phi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t off_psi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t off_sig[3] = {0, 0, 0};
    size_t off_flags = 0;
    size_t total = 0;
};

inline constexpr int kFlagBlocks = 1024;

// Deepest multi-step pass (levels per pass) of the 2D variants.
inline constexpr int kMaxLevels = 8;

// Levels per pass a variant asks for: TWOSTEP 2, THREESTEP 3, FOURSTEP 4,
// DEEP bits 20-23 of tile_rows (0: 6); 1 for the single-step variants.
inline int pass_depth(int variant, int tile_rows)
{
    switch (variant) {
    case DPML_VARIANT_TWOSTEP: return 2;
    case DPML_VARIANT_THREESTEP: return 3;
    case DPML_VARIANT_FOURSTEP: return 4;
    case DPML_VARIANT_DEEP: return ((tile_rows >> 20) & 0xF) ? ((tile_rows >> 20) & 0xF) : 6;
    default: return 1;
    }
}

template <typename V, int A, int B>
using Table2 = std::array<std::array<V, B>, A>;

template <typename V, int A, int B>
inline Table2<V, A, B> filled(V v)
{
    Table2<V, A, B> t;
    for (auto &r : t) r.fill(v);
    return t;
}

// U buffers of a single-grid handle: 2D grids carry kMaxLevels spares for
// the multi-step variants (which write U^{n+1} .. U^{n+levels} beside U^n
// and U^{n-1}); 3D grids two (U^{n+1}, U^{n+2} of the two-step pass).
inline int handle_ubufs(const dpml_grid_t *g) { return g && g->ndim == 2 ? 2 + kMaxLevels : 4; }

// Validate the grid and compute the workspace layout.  Returns "" or an error.
inline std::string make_layout(const dpml_grid_t *g, bool c2_field, Layout &L, int n_ubuf)
{
    if (!g) return "grid is NULL";
    if (g->ndim != 2 && g->ndim != 3) return "ndim must be 2 or 3";
    if (g->dtype != DPML_F32 && g->dtype != DPML_F64) return "dtype must be DPML_F32 or DPML_F64";
    L.ndim = g->ndim;
    L.dtype = g->dtype;
    L.esize = g->dtype == DPML_F32 ? 4 : 8;
    L.ncell = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < g->ndim) {
            if (g->n[a] < 1 || g->lo[a] < 0 || g->hi[a] < 0) return "extents must be n >= 1, lo, hi >= 0";
            L.n[a] = g->n[a];
            L.lo[a] = g->lo[a];
            L.hi[a] = g->hi[a];
            L.N[a] = g->n[a] + g->lo[a] + g->hi[a];
            if (L.N[a] < 3) return "each axis needs at least 3 cells";
            if (L.N[a] > (int64_t)1 << 30) return "axis too long";
            L.M[a] = g->lo[a] + g->hi[a];
            if (g->walls[a] != 0 && g->walls[a] != 1) return "walls[a] must be 0 or 1";
            L.wall[a] = g->walls[a];
        }
        L.ncell *= L.N[a];
    }
    L.batch = g->batch > 1 ? g->batch : 1;
    if (L.batch > 65535) return "batch too large";
    if (L.ncell * L.batch > ((int64_t)1 << 40)) return "grid too large";
    size_t off = 0;
    const size_t ubytes = align_up((size_t)(L.ncell * L.batch) * L.esize);
    L.n_ubuf = n_ubuf;
    for (int k = 0; k < n_ubuf; ++k) { L.off_u[k] = off; off += ubytes; }
    if (c2_field) { L.off_c2 = off; off += align_up((size_t)L.ncell * L.esize); }
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        L.aux_elems[a] = L.ncell / L.N[a] * (L.M[a] + 1);
        const size_t ab = align_up((size_t)(L.aux_elems[a] * L.batch) * L.esize);
        for (int k = 0; k < 2; ++k) {
            L.off_phi[a][k] = off; off += ab;
            L.off_psi[a][k] = off; off += ab;
        }
        L.off_sig[a] = off; off += align_up((size_t)(L.M[a] + 1) * L.esize);
    }
    L.off_flags = off; off += align_up(kFlagBlocks * sizeof(int32_t));
    L.total = off;
    return "";
}

using TileRefVec = std::vector<dpmlk::TileRef>;

}  // namespace dpmlh

struct dpml {
    using Layout = dpmlh::Layout;
    template <typename V, int A, int B> using Table2 = dpmlh::Table2<V, A, B>;
    Layout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    double h = 1, dt = 1;
    double c2_const = 1;     // used when c2 is not a field
    bool c2_field = false;
    void *u_now = nullptr, *u_old = nullptr;
    int cur = 0;             // aux buffer index holding time level n
    int64_t n = 0;
    bool state_set = false;
    int variant = DPML_VARIANT_AUTO;
    int tile_rows = 0;
    // frame tiles of the multi-step variants: [levels - 2][s] covers
    // everything outside the core shrunk by s cells (-1: not built yet)
    dpmlk::TileRef *d_frame[dpmlh::kMaxLevels - 1][dpmlh::kMaxLevels] = {};
    Table2<int64_t, dpmlh::kMaxLevels - 1, dpmlh::kMaxLevels> n_frame = dpmlh::filled<int64_t, dpmlh::kMaxLevels - 1, dpmlh::kMaxLevels>(-1);
    // the same frames as spans for the marching frame kernel (span rows fspan_rows)
    dpmlk::Span2 *d_fspan[dpmlh::kMaxLevels - 1][dpmlh::kMaxLevels] = {};
    Table2<int64_t, dpmlh::kMaxLevels - 1, dpmlh::kMaxLevels> n_fspan = dpmlh::filled<int64_t, dpmlh::kMaxLevels - 1, dpmlh::kMaxLevels>(-1);
    // tiles of the fused frame launch per depth ([levels - 2]; -1: not built yet)
    dpmlk::TileRef *d_ffused[dpmlh::kMaxLevels - 1] = {};
    int64_t n_ffused[dpmlh::kMaxLevels - 1] = {-1, -1, -1, -1, -1, -1, -1};
    int fspan_rows = 0;
    // the frame's steps run on a second stream beside the core kernel
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the adjoint's recompute beside its reverse sweep: a stream pair and
    // fork/join events of its own, and per history buffer the events that
    // order the two (recompute done, sweep done)
    hipStream_t adj_rs = nullptr, adj_rside = nullptr;
    hipEvent_t adj_rfork = nullptr, adj_rjoin = nullptr;
    hipEvent_t adj_rec_done[2] = {nullptr, nullptr}, adj_sweep_done[2] = {nullptr, nullptr};
    dpmlk::TileRef *d_adj_frame = nullptr;  // 2D adjoint: tiles outside the marching core
    int64_t n_adj_frame = -1;               // -1: not built yet
    dpmlk::TileRef *d_adj_frame_s[2] = {nullptr, nullptr};   // tiles outside the core shrunk by 1, 2
    int64_t n_adj_frame_s[2] = {-1, -1};
    int64_t *d_adj_frec_cells = nullptr;    // receivers the two-level pass's frame injects (sorted)
    int64_t *d_adj_frec_order = nullptr;
    int64_t n_adj_frec = -1;
    // sources
    int64_t ns = 0, nt_src = 0;
    int64_t *d_src_cells = nullptr, *d_src_order = nullptr;
    std::vector<int64_t> src_sorted;      // host copy of d_src_cells
    const void *wavelets = nullptr;
    // receivers
    int64_t nr = 0, nt_rec = 0;
    int64_t *d_rec_cells = nullptr;
    int64_t *d_rec_sorted = nullptr, *d_rec_order = nullptr;
    void *traces = nullptr;
    bool recording = true;   // off while the adjoint recomputes segments
    // checkpointed forward / adjoint
    char *adj_ws = nullptr;
    size_t adj_bytes = 0;
    int64_t adj_nsteps = 0, adj_every = 0;
    bool adj_ready = false;
    // cached HIP graph of a run of steps (no sources/receivers/planes)
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_steps = -1;
    int graph_cur = -1;
    void *graph_unow = nullptr, *graph_uold = nullptr;
    int graph_variant = -1, graph_rows = -1;
    void *graph_end_unow = nullptr, *graph_end_uold = nullptr;
    int graph_end_cur = 0;
    // RK4 integrator state (caller-owned workspace)
    char *rk_ws = nullptr;
    int rk_role[4] = {0, 1, 2, 3};   // buffer sets holding Y0, YS0, YS1, S
    int64_t rk_n = 0;
    bool rk_set = false;
    // plane recorder
    int plane_axis = -1;
    int64_t plane_index = 0, nt_plane = 0;
    void *planes = nullptr;
    // optional per-launch timing of the step kernels (event pairs on `stream`)
    struct Timed {
        int kind;
        hipEvent_t e0, e1;
        double bytes;
    };
    bool timing = false;
    std::vector<Timed> timed;
    std::vector<hipEvent_t> events;      // pool, reused after each dpml_get_timing
    size_t events_used = 0;
    std::string err;
    void *scratch = nullptr;   // this device's static scratch (dpml_step_checked_noalloc)
    // sources/receivers of the 2D multi-step passes: host copy of the
    // receivers, whether two share a cell (then no passes), the per-(member,
    // row) column maps, and per pass depth the receivers sorted by how deep
    // they lie in the core with the frame's share per level
    std::vector<int64_t> rec_host;
    bool rec_dups = false;
    int32_t *d_rmap = nullptr, *d_rpool = nullptr;
    int64_t *d_frec_cells[dpmlh::kMaxLevels - 1] = {};
    int32_t *d_frec_idx[dpmlh::kMaxLevels - 1] = {};
    std::array<int64_t, dpmlh::kMaxLevels + 1> frec_count[dpmlh::kMaxLevels - 1] = {};

    void *at(size_t off) { return ws + off; }
    int fail(int code, const std::string &msg) { err = msg; return code; }
};

namespace dpmlh {


inline int hip_fail(dpml *h, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (h) h->err = m; else g_create_error = m;
    return DPML_EHIP;
}

#define HIP_TRY(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

inline constexpr size_t kMaxTimed = 4096;    // launches recorded between two dpml_get_timing calls

// Layer axis-cells per member: M_a cells on every line along each axis a.
inline double aux_cells(const Layout &L)
{
    double aux = 0;
    for (int a = 0; a < L.ndim; ++a) aux += (double)L.M[a] * (double)(L.ncell / L.N[a]);
    return aux;
}

// Algorithmic bytes of one step over `cells` cells and `aux` layer
// axis-cells per member: 3 words per cell, 4 words per layer axis-cell and 1
// word per cell of a c^2 field.
inline double step_bytes(const dpml *H, double cells, double aux)
{
    const Layout &L = H->L;
    const double words = (3.0 * cells + 4.0 * aux) * (double)L.batch + (H->c2_field ? cells : 0.0);
    return words * (double)L.esize;
}

// Algorithmic bytes of the core launch of a multi-step pass over `cells`
// core cells per member: what the pass must move whatever its depth -- read
// U^n and U^{n-1}, write the pass's last two levels (4 words per cell), and
// 1 word per cell of a c^2 field.
inline double pass_bytes(const dpml *H, double cells)
{
    const Layout &L = H->L;
    const double words = 4.0 * cells * (double)L.batch + (H->c2_field ? cells : 0.0);
    return words * (double)L.esize;
}

inline hipEvent_t take_event(dpml *H)
{
    if (H->events_used == H->events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        H->events.push_back(e);
    }
    return H->events[H->events_used++];
}

// Record the start of a timed launch of class `kind` on stream s (default:
// the handle's); returns its slot or -1.
inline int timed_begin(dpml *H, int kind, double bytes, hipStream_t s = nullptr)
{
    if (!H->timing || H->timed.size() >= kMaxTimed) return -1;
    if (!s) s = H->stream;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(H->stream, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return -1;
    dpml::Timed t{kind, take_event(H), take_event(H), bytes};
    if (!t.e0 || !t.e1 || hipEventRecord(t.e0, s) != hipSuccess) return -1;
    H->timed.push_back(t);
    return (int)H->timed.size() - 1;
}

inline void timed_end(dpml *H, int slot, hipStream_t s = nullptr)
{
    if (slot >= 0) (void)hipEventRecord(H->timed[(size_t)slot].e1, s ? s : H->stream);
}

template <typename T>
inline dpmlk::Axis<T> make_axis(dpml *H, int a, bool next)
{
    dpmlk::Axis<T> A{};
    const Layout &L = H->L;
    A.N = (int32_t)L.N[a];
    A.b = (int32_t)(L.lo[a] + L.n[a]);
    A.M = a < L.ndim ? L.M[a] : 0;
    A.hi = L.hi[a];
    A.wall = a < L.ndim ? L.wall[a] : 0;
    if (A.M > 0) {
        const int in = H->cur, out = 1 - H->cur;
        A.sig = (const T *)H->at(L.off_sig[a]);
        A.phi = (const T *)H->at(L.off_phi[a][in]);
        A.psi = (const T *)H->at(L.off_psi[a][in]);
        A.phi_o = (T *)H->at(L.off_phi[a][out]);
        A.psi_o = (T *)H->at(L.off_psi[a][out]);
    }
    (void)next;
    return A;
}

template <typename T>
inline dpmlk::StepArgs<T> make_args(dpml *H)
{
    dpmlk::StepArgs<T> p{};
    const Layout &L = H->L;
    for (int a = 0; a < 3; ++a) p.ax[a] = make_axis<T>(H, a, true);
    p.u = (const T *)H->u_now;
    p.uo = (T *)H->u_old;
    p.c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
    p.c2_const = (T)H->c2_const;
    p.inv_h2 = (T)(1.0 / (H->h * H->h));
    p.inv_h = (T)(1.0 / H->h);
    p.inv_2h = (T)(1.0 / (2.0 * H->h));
    p.dt = (T)H->dt;
    p.dt2 = (T)(H->dt * H->dt);
    p.nx = (int32_t)L.N[0];
    p.ny = (int32_t)L.N[1];
    p.nz = (int32_t)L.N[2];
    p.bstride = L.ncell;
    for (int a = 0; a < 3; ++a) p.bstride_aux[a] = L.aux_elems[a];
    p.hist = nullptr;
    p.uout = nullptr;
    p.skip[0] = p.skip[1] = p.skip[2] = p.skip[3] = 0;
    return p;
}

template <typename T>
int launch_record(dpml *H, const T *unew, int64_t n);

inline int round8(int v) { return (v + 7) / 8 * 8; }

// The second stream (and its fork/join events) on which the layer parts of a
// split step run beside the main kernel.
inline int ensure_side(dpml *H)
{
    if (!H->side) HIP_TRY(H, hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking));
    if (!H->ev_fork) HIP_TRY(H, hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
    if (!H->ev_join) HIP_TRY(H, hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
    return DPML_OK;
}

template <typename T>
int launch_epilogue(dpml *H)
{
    // U^{n+1} now sits in u_old (before the rotation)
    T *unew = (T *)H->u_old;
    const Layout &L = H->L;
    if (H->ns > 0 && H->n < H->nt_src) {
        double hd = 1;
        for (int a = 0; a < L.ndim; ++a) hd *= H->h;
        const T amp = (T)(H->dt * H->dt / hd);
        dim3 grid((unsigned)((H->ns + 255) / 256)), block(256);
        hipLaunchKernelGGL((dpmlk::k_inject<T>), grid, block, 0, H->stream, unew, H->d_src_cells,
                           H->d_src_order, (const T *)H->wavelets, H->ns, H->nt_src, H->n, amp);
    }
    return launch_record<T>(H, unew, H->n);
}

// Receivers and the recorded plane of time index n from the field `unew`.
template <typename T>
int launch_record(dpml *H, const T *unew, int64_t n)
{
    const Layout &L = H->L;
    if (H->recording && H->nr > 0 && n < H->nt_rec) {
        dim3 grid((unsigned)((H->nr + 255) / 256)), block(256);
        hipLaunchKernelGGL((dpmlk::k_record<T>), grid, block, 0, H->stream, unew,
                           H->d_rec_cells, (T *)H->traces, H->nr, H->nt_rec, n);
    }
    if (H->recording && H->plane_axis >= 0 && n < H->nt_plane) {
        int a0 = -1, a1 = -1;
        for (int a = 0; a < L.ndim; ++a) {
            if (a == H->plane_axis) continue;
            if (a0 < 0) a0 = a; else a1 = a;
        }
        const int64_t stride[3] = {1, L.N[0], L.N[0] * L.N[1]};
        const int64_t e0 = L.N[a0], e1 = a1 >= 0 ? L.N[a1] : 1;
        const int64_t s0 = stride[a0], s1 = a1 >= 0 ? stride[a1] : 0;
        const int64_t cells = e0 * e1;
        T *out = (T *)H->planes + n * cells;
        dim3 grid((unsigned)((cells + 255) / 256)), block(256);
        hipLaunchKernelGGL((dpmlk::k_record_plane<T>), grid, block, 0, H->stream, unew, out,
                           e0, e1, s0, s1, H->plane_index * stride[H->plane_axis]);
    }
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}

// Multi-step passes with reflecting walls: the core kernels read `levels`
// cells beyond their outputs, which stays inside the grid (the ghost cells
// past a wall are never read) when every walled axis has a layer with at
// least one cell above the interior; an axis without a layer is core over its
// whole extent and wraps, so it must be periodic.
inline bool walls_allow_multistep(const Layout &L)
{
    for (int a = 0; a < L.ndim; ++a)
        if (L.wall[a] && (L.M[a] == 0 || L.N[a] - L.lo[a] - L.n[a] < 1)) return false;
    return true;
}

// Algorithmic layer axis-cells of a 3D box: per axis, the weight of each band
// slot in the box's range along it (a half word pair for each of Phi and Psi
// the slot holds, so a whole band counts M) times the box's other extents.
inline double box_aux(const Layout &L, const dpmlk::Box3 &bx)
{
    const int r0[3] = {bx.xs, bx.ys, bx.zs}, r1[3] = {bx.xe, bx.ye, bx.ze};
    double aux = 0;
    for (int a = 0; a < 3; ++a) {
        if (L.M[a] == 0) continue;
        const int64_t b = L.lo[a] + L.n[a], N = L.N[a];
        double w = 0;
        for (int i = r0[a]; i < r1[a]; ++i) {
            const int64_t ic = i % N;
            const int64_t j = ic >= b ? ic - b : ic + (N - b);
            if (j <= L.M[a]) w += 0.5 * ((j < L.M[a]) + (j > 0));
        }
        double other = 1;
        for (int c = 0; c < 3; ++c)
            if (c != a) other *= (double)(r1[c] - r0[c]);
        aux += w * other;
    }
    return aux;
}

inline double box_cells(const dpmlk::Box3 &bx)
{
    return (double)(bx.xe - bx.xs) * (double)(bx.ye - bx.ys) * (double)(bx.ze - bx.zs);
}

// ---- 3D stepping paths (dpml3d.hip; explicit instantiations for float and double)
// One 3D step by the marching kernels (variants MARCH/MARCH1 and the single
// steps of the multi-step variants): the step's U^{n+1} goes to p.uout (or
// over p.uo); sources/receivers are the caller's epilogue.
template <typename T>
int launch_march3d(dpml *H, dpmlk::StepArgs<T> p, int ry);

// Levels the next 3D pass may take (1: single steps).
int multistep_levels3d(const dpml *H, int64_t nsteps);

// One 3D multi-step pass (sources, receivers and plane included); advances
// the handle's time index by the pass's levels.
template <typename T>
int launch_multistep3d(dpml *H);

// The frame of a 3D two-step pass as two levels in one march per box
// (dpml_frame3d.hip): everything outside the core box c, as the seven boxes
// that lie outside c along a nonempty set of axes and inside its range
// along the others (each with the layer code of that set); U^{n+1} to out1,
// U^{n+2} to out2, the layer arrays of level n+2 to p's output aux buffers.
// `shape`: the launch shape bits of the pass's tile_rows; launches on st,
// the boxes outside c along two or three axes on st2 when shape asks for it.
template <typename T>
int launch_frame2_3d(dpml *H, const dpmlk::StepArgs<T> &p, T *out1, T *out2, const dpmlk::Box3 &c, int shape,
                     hipStream_t st, hipStream_t st2);

// ---- 2D history passes (dpml_hist.hip; explicit instantiations for float and double)
// The core kernel of a 2D pass of 4 .. kMaxLevels levels that stores every
// level: U^{n+l} (l < levels-1) at hist + (l-1) * hstride on the core cells
// at depth >= levels-l, the last two levels to pen and fin as the ordinary
// pass.  G: rows whose loads a wave issues together (1, 2 or 4).
template <typename T>
void launch_coreN_hist(int levels, int G, bool c2, dim3 grid, hipStream_t st, const dpmlk::StepArgs<T> &p, T *hist,
                       int64_t hstride, T *pen, T *fin, const int r[4], int strips, int n_waves,
                       const dpmlk::Taps2<T> &tp);

}  // namespace dpmlh

