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
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int ndim = 0;
    int dtype = 0;
    size_t esize = 0;
    int64_t N[3] = {1, 1, 1};
    int64_t n[3] = {1, 1, 1};
    int32_t lo[3] = {0, 0, 0};
    int32_t hi[3] = {0, 0, 0};
    int32_t M[3] = {0, 0, 0};
    int64_t ncell = 0;
    int64_t aux_elems[3] = {0, 0, 0};   // elements of one compact aux array
    // byte offsets into the workspace
    size_t off_u[2] = {0, 0};
    size_t off_c2 = 0;
    size_t off_phi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t off_psi[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    size_t off_sig[3] = {0, 0, 0};
    size_t off_flags = 0;
    size_t total = 0;
};

constexpr int kFlagBlocks = 1024;

// Validate the grid and compute the workspace layout.  Returns "" or an error.
std::string make_layout(const dpml_grid_t *g, bool c2_field, Layout &L)
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
        }
        L.ncell *= L.N[a];
    }
    if (L.ncell > ((int64_t)1 << 40)) return "grid too large";
    size_t off = 0;
    const size_t ubytes = align_up((size_t)L.ncell * L.esize);
    L.off_u[0] = off; off += ubytes;
    L.off_u[1] = off; off += ubytes;
    if (c2_field) { L.off_c2 = off; off += ubytes; }
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        L.aux_elems[a] = L.ncell / L.N[a] * (L.M[a] + 1);
        const size_t ab = align_up((size_t)L.aux_elems[a] * L.esize);
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

}  // namespace

struct dpml {
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
    // sources
    int64_t ns = 0, nt_src = 0;
    int64_t *d_src_cells = nullptr, *d_src_order = nullptr;
    const void *wavelets = nullptr;
    // receivers
    int64_t nr = 0, nt_rec = 0;
    int64_t *d_rec_cells = nullptr;
    void *traces = nullptr;
    // plane recorder
    int plane_axis = -1;
    int64_t plane_index = 0, nt_plane = 0;
    void *planes = nullptr;
    std::string err;

    void *at(size_t off) { return ws + off; }
    int fail(int code, const std::string &msg) { err = msg; return code; }
};

namespace {

int hip_fail(dpml *h, hipError_t e, const char *what)
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

template <typename T>
dpmlk::Axis<T> make_axis(dpml *H, int a, bool next)
{
    dpmlk::Axis<T> A{};
    const Layout &L = H->L;
    A.N = (int32_t)L.N[a];
    A.b = (int32_t)(L.lo[a] + L.n[a]);
    A.M = a < L.ndim ? L.M[a] : 0;
    A.hi = L.hi[a];
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
dpmlk::StepArgs<T> make_args(dpml *H)
{
    dpmlk::StepArgs<T> p{};
    const Layout &L = H->L;
    for (int a = 0; a < 3; ++a) p.ax[a] = make_axis<T>(H, a, true);
    p.u = (const T *)H->u_now;
    p.uo = (T *)H->u_old;
    p.c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
    const double kl = H->dt * H->dt / (H->h * H->h);
    p.k_lap = (T)(H->c2_field ? kl : kl * H->c2_const);
    p.k_damp = (T)(H->dt * H->dt / H->h);
    p.half_dt = (T)(0.5 * H->dt);
    p.dt_2h = (T)(H->dt / (2.0 * H->h));
    p.nx = (int32_t)L.N[0];
    p.ny = (int32_t)L.N[1];
    p.nz = (int32_t)L.N[2];
    return p;
}

int round8(int v) { return (v + 7) / 8 * 8; }

template <typename T>
int launch_step(dpml *H)
{
    const Layout &L = H->L;
    dpmlk::StepArgs<T> p = make_args<T>(H);
    int variant = H->variant == DPML_VARIANT_AUTO ? DPML_VARIANT_MARCH : H->variant;
    if (variant == DPML_VARIANT_CELL) {
        dim3 block(64, 4, 1);
        dim3 grid((unsigned)((L.N[0] + 63) / 64), (unsigned)((L.N[1] + 3) / 4),
                  (unsigned)(L.ndim == 3 ? L.N[2] : 1));
        if (L.ndim == 2)
            hipLaunchKernelGGL((dpmlk::k_step_cell<T, 2>), grid, block, 0, H->stream, p);
        else
            hipLaunchKernelGGL((dpmlk::k_step_cell<T, 3>), grid, block, 0, H->stream, p);
    } else if (L.ndim == 2) {
        // vector width: 8 bytes per thread when the rows allow it
        constexpr int VX = sizeof(T) == 4 ? 2 : 1;
        const int vx = (L.N[0] % VX == 0) ? VX : 1;
        p.tile_rows = H->tile_rows > 0 ? H->tile_rows : 32;
        p.tiles_x = (int)((L.N[0] + 256 * vx - 1) / (256 * vx));
        const int tiles_y = (int)((L.N[1] + p.tile_rows - 1) / p.tile_rows);
        p.n_tiles = p.tiles_x * tiles_y;
        dim3 grid((unsigned)round8(p.n_tiles)), block(256);
        if (vx == 2)
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, (sizeof(T) == 4 ? 2 : 1)>), grid, block, 0, H->stream, p);
        else
            hipLaunchKernelGGL((dpmlk::k_step_march2d<T, 1>), grid, block, 0, H->stream, p);
    } else {
        constexpr int RY = 2;
        p.tile_rows = H->tile_rows > 0 ? H->tile_rows : 40;
        p.tiles_x = (int)((L.N[0] + 63) / 64);
        p.tiles_y = (int)((L.N[1] + 4 * RY - 1) / (4 * RY));
        const int tiles_z = (int)((L.N[2] + p.tile_rows - 1) / p.tile_rows);
        p.n_tiles = p.tiles_x * p.tiles_y * tiles_z;
        dim3 grid((unsigned)round8(p.n_tiles)), block(64, 4);
        hipLaunchKernelGGL((dpmlk::k_step_march3d<T, RY>), grid, block, 0, H->stream, p);
    }
    HIP_TRY(H, hipGetLastError());
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
    if (H->nr > 0 && H->n < H->nt_rec) {
        dim3 grid((unsigned)((H->nr + 255) / 256)), block(256);
        hipLaunchKernelGGL((dpmlk::k_record<T>), grid, block, 0, H->stream, (const T *)unew,
                           H->d_rec_cells, (T *)H->traces, H->nr, H->nt_rec, H->n);
    }
    if (H->plane_axis >= 0 && H->n < H->nt_plane) {
        int a0 = -1, a1 = -1;
        for (int a = 0; a < L.ndim; ++a) {
            if (a == H->plane_axis) continue;
            if (a0 < 0) a0 = a; else a1 = a;
        }
        const int64_t stride[3] = {1, L.N[0], L.N[0] * L.N[1]};
        const int64_t e0 = L.N[a0], e1 = a1 >= 0 ? L.N[a1] : 1;
        const int64_t s0 = stride[a0], s1 = a1 >= 0 ? stride[a1] : 0;
        const int64_t cells = e0 * e1;
        T *out = (T *)H->planes + H->n * cells;
        dim3 grid((unsigned)((cells + 255) / 256)), block(256);
        hipLaunchKernelGGL((dpmlk::k_record_plane<T>), grid, block, 0, H->stream, (const T *)unew, out,
                           e0, e1, s0, s1, H->plane_index * stride[H->plane_axis]);
    }
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}

template <typename T>
int step_impl(dpml *H, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
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
    HIP_TRY(H, hipMemcpyAsync(H->u_now, U0, (size_t)L.ncell * sizeof(T), hipMemcpyDeviceToDevice, H->stream));
    for (int a = 0; a < L.ndim; ++a) {
        if (L.M[a] == 0) continue;
        for (int k = 0; k < 2; ++k) {
            HIP_TRY(H, hipMemsetAsync(H->at(L.off_phi[a][k]), 0, (size_t)L.aux_elems[a] * sizeof(T), H->stream));
            HIP_TRY(H, hipMemsetAsync(H->at(L.off_psi[a][k]), 0, (size_t)L.aux_elems[a] * sizeof(T), H->stream));
        }
    }
    const double kl = H->dt * H->dt / (H->h * H->h);
    const T half_k = (T)(0.5 * (H->c2_field ? kl : kl * H->c2_const));
    const T *c2 = H->c2_field ? (const T *)H->at(L.off_c2) : nullptr;
    dim3 block(64, 4, 1);
    dim3 grid((unsigned)((L.N[0] + 63) / 64), (unsigned)((L.N[1] + 3) / 4), (unsigned)(L.ndim == 3 ? L.N[2] : 1));
    // read U0 from the caller's buffer (the copy may still be in flight on the
    // same stream, which orders it before this kernel)
    if (L.ndim == 2)
        hipLaunchKernelGGL((dpmlk::k_start<T, 2>), grid, block, 0, H->stream, (const T *)U0, (const T *)V0,
                           (T *)H->u_old, c2, half_k, (T)H->dt, (int)L.N[0], (int)L.N[1], (int)L.N[2]);
    else
        hipLaunchKernelGGL((dpmlk::k_start<T, 3>), grid, block, 0, H->stream, (const T *)U0, (const T *)V0,
                           (T *)H->u_old, c2, half_k, (T)H->dt, (int)L.N[0], (int)L.N[1], (int)L.N[2]);
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

template <typename T>
int nonfinite_check(dpml *H, bool *bad)
{
    int32_t *flags = (int32_t *)H->at(H->L.off_flags);
    hipLaunchKernelGGL((dpmlk::k_nonfinite<T>), dim3(kFlagBlocks), dim3(256), 0, H->stream,
                       (const T *)H->u_now, H->L.ncell, flags);
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
    if (!make_layout(g, c2_is_field != 0, L).empty()) return 0;
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
    std::string e = make_layout(g, field, L);
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

    dpml *H = new (std::nothrow) dpml();
    if (!H) { g_create_error = "out of host memory"; return DPML_ENOMEM; }
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
        if (cells[s] < 0 || cells[s] >= H->L.ncell) return H->fail(DPML_EINVAL, "source cell out of range");
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    if (H->d_src_cells) { HIP_TRY(H, hipFree(H->d_src_cells)); H->d_src_cells = nullptr; }
    if (H->d_src_order) { HIP_TRY(H, hipFree(H->d_src_order)); H->d_src_order = nullptr; }
    H->ns = 0;
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
    return DPML_OK;
}

int dpml_record(dpml_t *H, int64_t nr, const int64_t *cells, void *traces, int64_t nt)
{
    if (!H) return DPML_EINVAL;
    if (nr < 0 || (nr > 0 && (!cells || !traces || nt < 1))) return H->fail(DPML_EINVAL, "bad receiver arguments");
    for (int64_t r = 0; r < nr; ++r)
        if (cells[r] < 0 || cells[r] >= H->L.ncell) return H->fail(DPML_EINVAL, "receiver cell out of range");
    HIP_TRY(H, hipStreamSynchronize(H->stream));
    if (H->d_rec_cells) { HIP_TRY(H, hipFree(H->d_rec_cells)); H->d_rec_cells = nullptr; }
    H->nr = 0;
    if (nr == 0) return DPML_OK;
    HIP_TRY(H, hipMalloc((void **)&H->d_rec_cells, (size_t)nr * sizeof(int64_t)));
    HIP_TRY(H, hipMemcpy(H->d_rec_cells, cells, (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice));
    H->nr = nr;
    H->nt_rec = nt;
    H->traces = traces;
    return DPML_OK;
}

int dpml_record_plane(dpml_t *H, int32_t axis, int64_t index, void *planes, int64_t nt)
{
    if (!H) return DPML_EINVAL;
    if (axis < 0) { H->plane_axis = -1; return DPML_OK; }
    if (axis >= H->L.ndim || index < 0 || index >= H->L.N[axis] || !planes || nt < 1)
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
    if (variant < DPML_VARIANT_AUTO || variant > DPML_VARIANT_MARCH || tile_rows < 0 || tile_rows > 4096)
        return H->fail(DPML_EINVAL, "bad variant");
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
    size_t b = 2 * (size_t)L.ncell * L.esize;
    for (int a = 0; a < L.ndim; ++a) b += 2 * (size_t)L.aux_elems[a] * L.esize;
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
    const size_t ub = (size_t)L.ncell * L.esize;
    int rc = cp(H->u_now, ub);
    if (!rc) rc = cp(H->u_old, ub);
    for (int a = 0; a < L.ndim && !rc; ++a) {
        if (L.M[a] == 0) continue;
        const size_t ab = (size_t)L.aux_elems[a] * L.esize;
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
                HIP_TRY(H, hipMemsetAsync(H->at(L.off_phi[a][k]), 0, (size_t)L.aux_elems[a] * L.esize, H->stream));
                HIP_TRY(H, hipMemsetAsync(H->at(L.off_psi[a][k]), 0, (size_t)L.aux_elems[a] * L.esize, H->stream));
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

void dpml_destroy(dpml_t *H)
{
    if (!H) return;
    (void)hipStreamSynchronize(H->stream);
    if (H->d_src_cells) (void)hipFree(H->d_src_cells);
    if (H->d_src_order) (void)hipFree(H->d_src_order);
    if (H->d_rec_cells) (void)hipFree(H->d_rec_cells);
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
