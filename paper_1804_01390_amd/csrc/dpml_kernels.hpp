// dpml_kernels.hpp -- gfx950 kernels of the discrete-PML wave stepper.
//
// One fused sweep per time step (Eq. (DiscretePML a-c), leapfrog for U and a
// forward step for Phi/Psi, every right-hand side from time level n):
//
//   U^{n+1}(i)  = 2U^n - U^{n-1} + dt^2 c^2 sum_a (U(i-e_a) - 2U + U(i+e_a))/h^2
//                 + dt^2/h sum_a ( sigma_a(i) Psi_a(i+e_a) - sigma_a(i-1) Phi_a(i-e_a) )
//   Phi_a^{n+1} = Phi_a - dt/2 (sigma_a(i-1) Phi_a(i-e_a) + sigma_a(i) Phi_a(i))
//                 - dt/(2h) (U(i+e_a) - U(i-e_a))
//   Psi_a^{n+1} = Psi_a - dt/2 (sigma_a(i-1) Psi_a(i) + sigma_a(i) Psi_a(i+e_a))
//                 - dt/(2h) (U(i+e_a) - U(i-e_a))
//
// Every expression is evaluated in the plain order of the equations (sum
// over axes x, y, z; no contraction into FMAs: the library is compiled with
// -ffp-contract=off), so with h and dt powers of two the FP64 results do not
// depend on how the sweep is tiled.
//
// U^{n+1} overwrites U^{n-1} in place (each cell reads its own old value
// before writing it; neighbours are read from U^n only).  Phi/Psi are double
// buffered because the update of band slot j reads slots j-1 / j+1.
//
// Layout: x fastest.  The layer along axis a is the periodic band
// [b, N) U [0, lo) with b = lo + n; its band coordinate is
// j = (i - b) mod N in [0, M], M = lo + hi, and Phi_a/Psi_a are stored
// compactly with extent M+1 in place of N along axis a.  The damping table
// sig[j] holds sigma_a at array index (b + j) mod N (sig[M] = sigma(lo) = 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpmlk {

template <typename T>
struct Axis {
    int32_t N;        // cells along the axis
    int32_t b;        // first band cell (lo + n)
    int32_t M;        // band thickness lo + hi (0: no layer on this axis)
    int32_t hi;       // N - b
    int32_t wall;     // 0: periodic; 1: reflecting walls (ghost cells -1, N hold 0)
    int32_t pad_;
    const T *sig;     // sig[j], j in [0, M]
    const T *phi;     // Phi_a^n   (compact)
    const T *psi;     // Psi_a^n   (compact)
    T *phi_o;         // Phi_a^{n+1}
    T *psi_o;         // Psi_a^{n+1}
};

template <typename T>
struct StepArgs {
    Axis<T> ax[3];
    const T *u;       // U^n
    T *uo;            // U^{n-1} on entry, U^{n+1} on exit
    const T *c2;      // per-cell c^2, or nullptr
    T c2_const;       // c^2 when c2 == nullptr
    T inv_h2;         // 1 / h^2
    T inv_h;          // 1 / h
    T inv_2h;         // 1 / (2h)
    T dt;             // dt
    T dt2;            // dt * dt
    int32_t nx, ny, nz;
    int32_t tiles_x;  // tiles along x (marching kernels)
    int32_t tiles_y;  // tiles along y (3D marching kernel)
    int32_t tile_rows;// rows (2D) or planes (3D) per marching tile
    int32_t n_tiles;  // real tiles (the grid may be padded to a multiple of 8)
    int64_t bstride;  // elements between batch members in U
    int64_t bstride_aux[3];  // elements between batch members in Phi_a/Psi_a
    T *hist;          // optional: also store U^{n+1} here (same layout as U), or nullptr
    T *uout;          // optional: write U^{n+1} here instead of over U^{n-1}
    int32_t skip[4];  // cells with skip[0] <= x < skip[1], skip[2] <= y < skip[3] are left alone
};

// Point the step arguments at batch member bi.
template <typename T>
__device__ __forceinline__ void select_member(StepArgs<T> &p, int bi)
{
    const int64_t o = (int64_t)bi * p.bstride;
    p.u += o;
    p.uo += o;
    if (p.hist) p.hist += o;
    if (p.uout) p.uout += o;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t oa = (int64_t)bi * p.bstride_aux[a];
        p.ax[a].phi += oa;
        p.ax[a].psi += oa;
        p.ax[a].phi_o += oa;
        p.ax[a].psi_o += oa;
    }
}

struct TileRef {
    int32_t prob, tx, ty, pad;
};

__device__ __forceinline__ int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// Band coordinate of array index i along an axis, or a value > M outside the
// band and the first interior cell.
template <typename T>
__device__ __forceinline__ int band_coord(const Axis<T> &A, int i)
{
    return i >= A.b ? i - A.b : i + A.hi;
}

// Damping terms of one axis at a cell with band coordinate j <= M (Eqs.
// (DiscretePML b, c) with a forward step):
//   Phi' = Phi + dt (-1/2 (sigma(i-1) Phi(i-e) + sigma(i) Phi) - (U(i+e) - U(i-e))/(2h))
//   Psi' = Psi + dt (-1/2 (sigma(i-1) Psi + sigma(i) Psi(i+e)) - (U(i+e) - U(i-e))/(2h))
// and the contribution sigma(i) Psi(i+e) - sigma(i-1) Phi(i-e) to Eq.
// (DiscretePML a) (to be scaled by 1/h).  Split in two: layer_load reads
// everything one axis needs, layer_finish computes and stores; a cell
// issues the loads of all its axes before the first store, so the (possibly
// aliasing) stores of one axis do not hold back the loads of the next.
// um, up = U(i-e), U(i+e).
template <typename T>
struct LayerIn {
    T s, sl, phi_l, psi_r, phi_c, psi_c;
    int64_t c;
    bool on;          // the cell has this axis's terms (j <= M)
};

// Axis a's compact index of slot 0 for the line through (x, y, z), and the
// axis's stride in the compact array.
template <int A_>
__device__ __forceinline__ int64_t layer_base(int M, int64_t nx, int64_t ny, int x, int y, int z)
{
    if (A_ == 0) return ((int64_t)z * ny + y) * (M + 1);      // [z][y][Mx+1]
    if (A_ == 1) return (int64_t)z * (M + 1) * nx + x;         // [z][My+1][x]
    return (int64_t)y * nx + x;                                // [Mz+1][y][x]
}

template <int A_, typename T>
__device__ __forceinline__ LayerIn<T> layer_load(const Axis<T> &A, int j, int64_t nx, int64_t ny, int x, int y,
                                                 int z)
{
    LayerIn<T> L;
    L.on = j <= A.M;
    L.s = L.sl = L.phi_l = L.psi_r = L.phi_c = L.psi_c = T(0);
    L.c = 0;
    if (!L.on) return L;
    const int64_t cstr = A_ == 0 ? 1 : (A_ == 1 ? nx : nx * ny);
    L.c = layer_base<A_>(A.M, nx, ny, x, y, z) + (int64_t)j * cstr;
    // with walls, slot hi is cell 0 (its left neighbour is a ghost and the
    // ghost edge is undamped) and slot hi-1 is cell N-1 (right neighbour ghost)
    const bool left_ghost = A.wall && j == A.hi;
    const bool right_ghost = A.wall && j == A.hi - 1;
    L.s = A.sig[j];                                                      // sigma_a(i)
    if (j > 0 && !left_ghost) {
        L.sl = A.sig[j - 1];                                             // sigma_a(i-1)
        L.phi_l = A.phi[L.c - cstr];                                     // Phi_a(i-e)
    }
    if (j < A.M && !right_ghost) L.psi_r = A.psi[L.c + cstr];           // Psi_a(i+e)
    if (j < A.M) L.phi_c = A.phi[L.c];
    if (j > 0) L.psi_c = A.psi[L.c];
    return L;
}

template <typename T>
__device__ __forceinline__ T layer_finish(const Axis<T> &A, const LayerIn<T> &L, int j, T um, T up, T dt, T inv_2h)
{
    // (L.c is only meaningful when L.on; callers test it)
    const T grad = (up - um) * inv_2h;
    if (j < A.M) A.phi_o[L.c] = L.phi_c + dt * (T(-0.5) * (L.sl * L.phi_l + L.s * L.phi_c) - grad);
    if (j > 0) A.psi_o[L.c] = L.psi_c + dt * (T(-0.5) * (L.sl * L.psi_c + L.s * L.psi_r) - grad);
    return L.s * L.psi_r - L.sl * L.phi_l;
}

// The same terms in one piece (loads, arithmetic and stores of one axis
// together): fewer instructions and registers where most cells lie off the
// layer.
template <int A_, typename T>
__device__ __forceinline__ T layer_terms(const Axis<T> &A, int j, int64_t nx, int64_t ny, int x, int y, int z,
                                         T um, T up, T dt, T inv_2h)
{
    const int64_t cstr = A_ == 0 ? 1 : (A_ == 1 ? nx : nx * ny);
    const int64_t c = layer_base<A_>(A.M, nx, ny, x, y, z) + (int64_t)j * cstr;
    const bool left_ghost = A.wall && j == A.hi;
    const bool right_ghost = A.wall && j == A.hi - 1;
    const T s = A.sig[j];                                              // sigma_a(i)
    const T sl = (j > 0 && !left_ghost) ? A.sig[j - 1] : T(0);         // sigma_a(i-1)
    const T phi_l = (j > 0 && !left_ghost) ? A.phi[c - cstr] : T(0);   // Phi_a(i-e)
    const T psi_r = (j < A.M && !right_ghost) ? A.psi[c + cstr] : T(0); // Psi_a(i+e)
    const T grad = (up - um) * inv_2h;
    if (j < A.M) {
        const T phi_c = A.phi[c];
        A.phi_o[c] = phi_c + dt * (T(-0.5) * (sl * phi_l + s * phi_c) - grad);
    }
    if (j > 0) {
        const T psi_c = A.psi[c];
        A.psi_o[c] = psi_c + dt * (T(-0.5) * (sl * psi_c + s * psi_r) - grad);
    }
    return s * psi_r - sl * phi_l;
}

// Complete update of one cell given its stencil values.  (x, y, z) are the
// cell coordinates; for 2D z = 0 and the z values are unused.  AX is the set
// of axes (bit a for axis a) whose layer terms the caller may meet; the
// others are left out of the code (callers that only see cells off those
// bands).  HOIST: issue the layer loads of all axes before any of their
// stores (kernels whose cells mostly lie in the layer); otherwise each
// axis's terms are evaluated in one piece (kernels whose cells mostly lie
// off it).  Both evaluate the same expressions in the same order.
template <typename T, int D, int AX = 7, bool HOIST = false>
__device__ __forceinline__ T cell_update(const StepArgs<T> &p, int x, int y, int z, int64_t idx,
                                         T uc, T uxm, T uxp, T uym, T uyp, T uzm, T uzp, T uold)
{
    const int64_t nx = p.nx, ny = p.ny;
    if (!HOIST) {
        // Eq. (DiscretePML a): c^2 sum_a (U(i-e) - 2U + U(i+e))/h^2 + sum_a (...)/h
        T lap = ((uxm - T(2) * uc) + uxp) * p.inv_h2;
        lap += ((uym - T(2) * uc) + uyp) * p.inv_h2;
        if (D == 3) lap += ((uzm - T(2) * uc) + uzp) * p.inv_h2;
        const T c2 = p.c2 ? p.c2[idx] : p.c2_const;
        T damp = T(0);
        if ((AX & 1) && p.ax[0].M > 0) {
            const int j = band_coord(p.ax[0], x);
            if (j <= p.ax[0].M) damp += layer_terms<0>(p.ax[0], j, nx, ny, x, y, z, uxm, uxp, p.dt, p.inv_2h) * p.inv_h;
        }
        if ((AX & 2) && p.ax[1].M > 0) {
            const int j = band_coord(p.ax[1], y);
            if (j <= p.ax[1].M) damp += layer_terms<1>(p.ax[1], j, nx, ny, x, y, z, uym, uyp, p.dt, p.inv_2h) * p.inv_h;
        }
        if (D == 3 && (AX & 4) && p.ax[2].M > 0) {
            const int j = band_coord(p.ax[2], z);
            if (j <= p.ax[2].M) damp += layer_terms<2>(p.ax[2], j, nx, ny, x, y, z, uzm, uzp, p.dt, p.inv_2h) * p.inv_h;
        }
        const T rhs = c2 * lap + damp;
        return (T(2) * uc - uold) + p.dt2 * rhs;
    }
    // loads first: c^2 and the layer inputs of every axis
    const T c2 = p.c2 ? p.c2[idx] : p.c2_const;
    const bool lx = (AX & 1) && p.ax[0].M > 0, ly = (AX & 2) && p.ax[1].M > 0;
    const bool lz = D == 3 && (AX & 4) && p.ax[2].M > 0;
    int jx = 0, jy = 0, jz = 0;
    LayerIn<T> Lx, Ly, Lz;
    Lx.on = Ly.on = Lz.on = false;
    if (lx) {
        jx = band_coord(p.ax[0], x);
        Lx = layer_load<0>(p.ax[0], jx, nx, ny, x, y, z);
    }
    if (ly) {
        jy = band_coord(p.ax[1], y);
        Ly = layer_load<1>(p.ax[1], jy, nx, ny, x, y, z);
    }
    if (lz) {
        jz = band_coord(p.ax[2], z);
        Lz = layer_load<2>(p.ax[2], jz, nx, ny, x, y, z);
    }
    // Eq. (DiscretePML a): c^2 sum_a (U(i-e) - 2U + U(i+e))/h^2 + sum_a (...)/h
    T lap = ((uxm - T(2) * uc) + uxp) * p.inv_h2;
    lap += ((uym - T(2) * uc) + uyp) * p.inv_h2;
    if (D == 3) lap += ((uzm - T(2) * uc) + uzp) * p.inv_h2;
    T damp = T(0);
    if (lx && Lx.on) damp += layer_finish(p.ax[0], Lx, jx, uxm, uxp, p.dt, p.inv_2h) * p.inv_h;
    if (ly && Ly.on) damp += layer_finish(p.ax[1], Ly, jy, uym, uyp, p.dt, p.inv_2h) * p.inv_h;
    if (lz && Lz.on) damp += layer_finish(p.ax[2], Lz, jz, uzm, uzp, p.dt, p.inv_2h) * p.inv_h;
    const T rhs = c2 * lap + damp;
    return (T(2) * uc - uold) + p.dt2 * rhs;
}

// Map a hardware block id to a logical tile so that the blocks one XCD
// executes (ids congruent mod 8) get consecutive tiles: neighbouring tiles
// then share their halo rows in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks >> 3;   // nblocks is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Variant CELL: one thread per cell; a block of 256 threads covers a
// (256/TH) x TH tile of an (x, y) row band.  The launch is 1-D and goes
// through xcd_tile, so the tiles one XCD runs are consecutive in row-major
// tile order: a tile's halo rows are read by its vertical neighbours on the
// same XCD at nearly the same time and are served by that XCD's L2.
// ---------------------------------------------------------------------------
template <typename T, int D, int TH>
__global__ void __launch_bounds__(256) k_step_cell(StepArgs<T> p)
{
    constexpr int TW = 256 / TH;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
    select_member(p, (int)blockIdx.y);
    const int per_plane = p.tiles_x * p.tiles_y;
    const int z = D == 3 ? tile / per_plane : 0;
    const int rem = tile - z * per_plane;
    const int ty = rem / p.tiles_x;
    const int tx = rem - ty * p.tiles_x;
    const int x = tx * TW + (int)(threadIdx.x % TW);
    const int y = ty * TH + (int)(threadIdx.x / TW);
    if (x >= p.nx || y >= p.ny) return;
    const int64_t nx = p.nx, ny = p.ny;
    const int64_t row = ((int64_t)z * ny + y) * nx;
    const int64_t idx = row + x;
    const T *u = p.u;
    const int xm = wrap_dec(x, p.nx), xp = wrap_inc(x, p.nx);
    const int ym = wrap_dec(y, p.ny), yp = wrap_inc(y, p.ny);
    T uzm = T(0), uzp = T(0);
    if (D == 3) {
        const int zm = wrap_dec(z, p.nz), zp = wrap_inc(z, p.nz);
        uzm = (p.ax[2].wall && z == 0) ? T(0) : u[((int64_t)zm * ny + y) * nx + x];
        uzp = (p.ax[2].wall && z == p.nz - 1) ? T(0) : u[((int64_t)zp * ny + y) * nx + x];
    }
    const int64_t plane = (int64_t)z * ny * nx;
    const T uxm = (p.ax[0].wall && x == 0) ? T(0) : u[row + xm];
    const T uxp = (p.ax[0].wall && x == p.nx - 1) ? T(0) : u[row + xp];
    const T uym = (p.ax[1].wall && y == 0) ? T(0) : u[plane + (int64_t)ym * nx + x];
    const T uyp = (p.ax[1].wall && y == p.ny - 1) ? T(0) : u[plane + (int64_t)yp * nx + x];
    const T r = cell_update<T, D>(p, x, y, z, idx, u[idx], uxm, uxp, uym, uyp, uzm, uzp, p.uo[idx]);
    (p.uout ? p.uout : p.uo)[idx] = r;
    if (p.hist) p.hist[idx] = r;
}

// ---------------------------------------------------------------------------
// Variant MARCH, 2D: a block of 256 threads owns 256*VX consecutive columns
// and marches over `tile_rows` rows, keeping U^n of rows y-1, y, y+1 in
// registers.  Each row of U^n is read from HBM once per tile (plus two halo
// rows per tile); x neighbours inside the thread's vector come from
// registers, the two outer ones from the L1 cache.
// ---------------------------------------------------------------------------
template <typename T, int VX> struct Vec;
template <> struct Vec<float, 1> { using type = float; };
template <> struct Vec<float, 2> { using type = float2; };
template <> struct Vec<float, 4> { using type = float4; };
template <> struct Vec<double, 1> { using type = double; };
template <> struct Vec<double, 2> { using type = double2; };

template <typename T, int VX>
struct Row {
    T v[VX];
};

template <typename T, int VX>
__device__ __forceinline__ Row<T, VX> load_row(const T *ptr)
{
    Row<T, VX> r;
    using V = typename Vec<T, VX>::type;
    const V w = *reinterpret_cast<const V *>(ptr);
    const T *e = reinterpret_cast<const T *>(&w);
#pragma unroll
    for (int k = 0; k < VX; ++k) r.v[k] = e[k];
    return r;
}

template <typename T, int VX>
__device__ __forceinline__ void store_row(T *ptr, const Row<T, VX> &r)
{
    using V = typename Vec<T, VX>::type;
    V w;
    T *e = reinterpret_cast<T *>(&w);
#pragma unroll
    for (int k = 0; k < VX; ++k) e[k] = r.v[k];
    *reinterpret_cast<V *>(ptr) = w;
}

// One 2D marching tile (tile column tx, tile row ty) of one problem.  The
// thread keeps a window of U^n rows in registers and walks down the tile in
// groups of R rows: all HBM loads of a group (R new U^n rows, R U^{n-1}
// rows, and the 2R outer x neighbours, which hit L1) are issued before any
// of its arithmetic, so each wave has R times more loads in flight than a
// row-at-a-time loop.  Register arrays are only indexed with compile-time
// constants (full groups); the last rows of a tile take a one-row loop.
template <typename T, int VX, int R, bool HOIST = false, int AX = 7>
__device__ __forceinline__ void march2d_tile(const StepArgs<T> &p, int tx, int ty)
{
    const int x0 = (tx * 256 + (int)threadIdx.x) * VX;
    if (x0 >= p.nx) return;
    const int nx = p.nx, ny = p.ny;
    const int y0 = ty * p.tile_rows;
    const int y1 = min(y0 + p.tile_rows, ny);
    const T *u = p.u;
    const int xl = wrap_dec(x0, nx);          // left neighbour of the vector
    const int xr = wrap_inc(x0 + VX - 1, nx); // right neighbour of the vector
    const bool lghost = p.ax[0].wall && x0 == 0;
    const bool rghost = p.ax[0].wall && x0 + VX == nx;
    const bool wy = p.ax[1].wall;
    // row yy of U^n (a zero row past a wall)
    auto nb_row = [&](int yy) -> Row<T, VX> {
        if (wy && (yy < 0 || yy >= ny)) {
            Row<T, VX> z;
#pragma unroll
            for (int k = 0; k < VX; ++k) z.v[k] = T(0);
            return z;
        }
        const int w = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        return load_row<T, VX>(u + (int64_t)w * nx + x0);
    };
    auto row_out = [&](int y, const Row<T, VX> &um, const Row<T, VX> &uc, const Row<T, VX> &up,
                       const Row<T, VX> &old, T left, T right) {
        const int64_t row = (int64_t)y * nx;
        Row<T, VX> out;
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const T uxm = k == 0 ? left : uc.v[k - 1];
            const T uxp = k == VX - 1 ? right : uc.v[k + 1];
            out.v[k] = cell_update<T, 2, AX, HOIST>(p, x0 + k, y, 0, row + x0 + k, uc.v[k], uxm, uxp,
                                          um.v[k], up.v[k], T(0), T(0), old.v[k]);
        }
        store_row<T, VX>((p.uout ? p.uout : p.uo) + row + x0, out);
        if (p.hist) store_row<T, VX>(p.hist + row + x0, out);
    };

    Row<T, VX> w[R + 2];       // w[0] = row y-1, w[1] = row y, w[2 + r] = row y+1+r
    w[0] = nb_row(y0 - 1);
    w[1] = load_row<T, VX>(u + (int64_t)y0 * nx + x0);
    int y = y0;
    for (; y + R <= y1; y += R) {
        Row<T, VX> old[R];
        T left[R], right[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = (int64_t)(y + r) * nx;
            w[2 + r] = nb_row(y + 1 + r);
            old[r] = load_row<T, VX>(p.uo + row + x0);
            left[r] = lghost ? T(0) : u[row + xl];
            right[r] = rghost ? T(0) : u[row + xr];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) row_out(y + r, w[r], w[r + 1], w[r + 2], old[r], left[r], right[r]);
        w[0] = w[R];
        w[1] = w[R + 1];
    }
    for (; y < y1; ++y) {
        const int64_t row = (int64_t)y * nx;
        w[2] = nb_row(y + 1);
        const Row<T, VX> old = load_row<T, VX>(p.uo + row + x0);
        const T left = lghost ? T(0) : u[row + xl];
        const T right = rghost ? T(0) : u[row + xr];
        row_out(y, w[0], w[1], w[2], old, left, right);
        w[0] = w[1];
        w[1] = w[2];
    }
}

template <typename T, int VX, int R>
__global__ void __launch_bounds__(256) k_step_march2d(StepArgs<T> p)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
    select_member(p, (int)blockIdx.y);
    march2d_tile<T, VX, R>(p, tile % p.tiles_x, tile / p.tiles_x);
}

// One (256/TH) x TH cell tile of a 2D problem, one thread per cell, with
// the layer loads hoisted (the body of the frame kernels, whose cells mostly
// lie in the layer).
template <typename T, int TH>
__device__ __forceinline__ void cell2d_tile(const StepArgs<T> &p, int tx, int ty)
{
    constexpr int TW = 256 / TH;
    const int x = tx * TW + (int)(threadIdx.x % TW);
    const int y = ty * TH + (int)(threadIdx.x / TW);
    if (x >= p.nx || y >= p.ny) return;
    const int64_t nx = p.nx;
    const int64_t row = (int64_t)y * nx;
    const int64_t idx = row + x;
    const T *u = p.u;
    const int xm = wrap_dec(x, p.nx), xp = wrap_inc(x, p.nx);
    const int ym = wrap_dec(y, p.ny), yp = wrap_inc(y, p.ny);
    const T uxm = (p.ax[0].wall && x == 0) ? T(0) : u[row + xm];
    const T uxp = (p.ax[0].wall && x == p.nx - 1) ? T(0) : u[row + xp];
    const T uym = (p.ax[1].wall && y == 0) ? T(0) : u[(int64_t)ym * nx + x];
    const T uyp = (p.ax[1].wall && y == p.ny - 1) ? T(0) : u[(int64_t)yp * nx + x];
    const T r = cell_update<T, 2, 7, true>(p, x, y, 0, idx, u[idx], uxm, uxp, uym, uyp, T(0), T(0), p.uo[idx]);
    (p.uout ? p.uout : p.uo)[idx] = r;
    if (p.hist) p.hist[idx] = r;
}

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking), 2D, periodic grids.
//
// The "core" -- cells whose one-cell halo lies where no damping term acts,
// inside [lo+2, lo+n-1) per axis -- advances two levels in one pass.  Each
// wave works alone (no barriers, no LDS): it owns a strip of 64 lanes x VX
// columns, lanes 1..62 produce output and lanes 0 and 63 carry the halo, and
// it marches down a tile of rows.  For every row r it reads U^n(r+1) and
// U^{n-1}(r), computes U^{n+1}(r) and then U^{n+2}(r-1) from the three newest
// U^{n+1} rows held in registers; x neighbours across lanes come from
// cross-lane shuffles.  Reads U^n, U^{n-1}; writes U^{n+1}, U^{n+2} (into two
// further buffers): 2 words per cell per step instead of 3.
//
// The frame (everything outside the core, layer included) advances by
// ordinary steps on a second stream at the same time: its first step also
// covers the core's one-cell boundary ring, so the core leaves U^{n+1} there
// to it (store_inner) and the two never write the same cell.  The core
// evaluates the scheme in the operation order of cell_update (no damping
// terms there), so results are bit-identical to single steps.
// ---------------------------------------------------------------------------
// Whole-wave shifts by one lane through DPP (a modifier on a VALU move, no
// LDS round trip): lane i receives lane i-1's value (from_left) or lane
// i+1's (from_right); the lane with no source keeps its own value.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_shift(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_move<CTRL>(__builtin_bit_cast(int, v)));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)dpp_move<CTRL>((int)(uint32_t)b);
        const uint32_t hi = (uint32_t)dpp_move<CTRL>((int)(uint32_t)(b >> 32));
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_shift<0x138>(v); }    // wave_shr:1

template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_shift<0x130>(v); }   // wave_shl:1

template <typename T, int VX, bool C2F>
struct March2Ctx {
    using R = Row<T, VX>;
    const T *u, *up, *c2;          // U^n, U^{n-1}, c^2 field
    T *o1, *o2;                    // U^{n+1}, U^{n+2}
    T inv_h2, dt2, c2c;
    int nx, ny, xs, xw, cx0, cx1, cy0, cy1;
    bool need, vec, out;

    // store of a row that leaves the core's boundary ring (first/last row and
    // column of the core) alone: the frame steps own those cells there
    __device__ __forceinline__ void store_inner(T *f, int y, const R &r) const
    {
        if (!out || y == cy0 || y == cy1 - 1) return;
        T *row = f + (int64_t)y * nx + xs;
        if (xs > cx0 && xs + VX < cx1) {
            store_row<T, VX>(row, r);
        } else {
#pragma unroll
            for (int k = 0; k < VX; ++k)
                if (xs + k > cx0 && xs + k < cx1 - 1) row[k] = r.v[k];
        }
    }

    __device__ __forceinline__ int wrapy(int y) const { return y < 0 ? y + ny : (y >= ny ? y - ny : y); }

    // this lane's VX cells of row y of field f (row index already wrapped)
    __device__ __forceinline__ R load(const T *f, int y) const
    {
        R r;
        const T *row = f + (int64_t)y * nx;
        if (!need) {
#pragma unroll
            for (int k = 0; k < VX; ++k) r.v[k] = T(0);
        } else if (vec) {
            r = load_row<T, VX>(row + xw);
        } else {
#pragma unroll
            for (int k = 0; k < VX; ++k) {
                int x = (xs + k) % nx;
                if (x < 0) x += nx;
                r.v[k] = row[x];
            }
        }
        return r;
    }

    __device__ __forceinline__ void store(T *f, int y, const R &r) const
    {
        if (!out) return;
        T *row = f + (int64_t)y * nx + xs;
        if (xs + VX <= cx1) {
            store_row<T, VX>(row, r);
        } else {
#pragma unroll
            for (int k = 0; k < VX; ++k)
                if (xs + k < cx1) row[k] = r.v[k];
        }
    }

    // one undamped leapfrog level for this lane's cells (Eq. (DiscretePML a)
    // with every damping term zero), in cell_update's operation order
    __device__ __forceinline__ R level(const R &um, const R &uc, const R &upr, const R &old, const R &c) const
    {
        const T left = from_left(uc.v[VX - 1]);
        const T right = from_right(uc.v[0]);
        R o;
#pragma unroll
        for (int k = 0; k < VX; ++k) {
            const T uxm = k == 0 ? left : uc.v[k - 1];
            const T uxp = k == VX - 1 ? right : uc.v[k + 1];
            T lap = ((uxm - T(2) * uc.v[k]) + uxp) * inv_h2;
            lap += ((um.v[k] - T(2) * uc.v[k]) + upr.v[k]) * inv_h2;
            const T cc = C2F ? c.v[k] : c2c;
            o.v[k] = (T(2) * uc.v[k] - old.v[k]) + dt2 * (cc * lap);
        }
        return o;
    }

    // A tile's rows are visited in march order k = 0, 1, ..., L-1 (L rows):
    // row base + DIR k.  Odd tile rows march upwards (DIR = -1), so two
    // neighbouring tiles reach their shared halo rows at the same time (both
    // at the start, or both at the end) and the second read hits the L2.
    // level() takes rows in grid order (y-1, y, y+1), whatever DIR is.
    template <int DIR>
    __device__ __forceinline__ R lev(const R &prev, const R &cur, const R &next, const R &old, const R &c) const
    {
        return DIR > 0 ? level(prev, cur, next, old, c) : level(next, cur, prev, old, c);
    }

    // rolling state at march index k: U^n at k-1, k; U^{n+1} at k-2, k-1; c^2 at k-1
    struct State {
        R n0, n1, v0, v1, c0;
    };

    // U^{n+1} at march indices k .. k+G-1 and U^{n+2} at k-1 .. k+G-2; every
    // load of the group is issued before its arithmetic
    template <int G, int DIR>
    __device__ __forceinline__ void group(State &s, int base, int k, int L) const
    {
        R wn[G + 2], po[G], v[G + 2], cw[G + 1];
        wn[0] = s.n0;
        wn[1] = s.n1;
        v[0] = s.v0;
        v[1] = s.v1;
        cw[0] = s.c0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            wn[2 + g] = load(u, wrapy(base + DIR * (k + 1 + g)));
            po[g] = load(up, wrapy(base + DIR * (k + g)));
            if (C2F) cw[1 + g] = load(c2, wrapy(base + DIR * (k + g)));
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            v[2 + g] = lev<DIR>(wn[g], wn[g + 1], wn[g + 2], po[g], cw[1 + g]);
            if (k + g < L) store_inner(o1, base + DIR * (k + g), v[2 + g]);
            store(o2, base + DIR * (k - 1 + g), lev<DIR>(v[g], v[g + 1], v[g + 2], wn[g], cw[g]));
        }
        s.n0 = wn[G];
        s.n1 = wn[G + 1];
        s.v0 = v[G];
        s.v1 = v[G + 1];
        s.c0 = cw[G];
    }

    // the whole tile: rows base, base + DIR, ..., L rows
    template <int G, int DIR>
    __device__ __forceinline__ void march(int base, int L) const
    {
        State s;
        {
            // U^{n+1} at march indices -1 and 0
            const R a0 = load(u, wrapy(base - 2 * DIR)), a1 = load(u, wrapy(base - DIR));
            const R a2 = load(u, base), a3 = load(u, wrapy(base + DIR));
            const R p0 = load(up, wrapy(base - DIR)), p1 = load(up, base);
            R k0{}, k1{};
            if (C2F) {
                k0 = load(c2, wrapy(base - DIR));
                k1 = load(c2, base);
            }
            s.v0 = lev<DIR>(a0, a1, a2, p0, k0);
            s.v1 = lev<DIR>(a1, a2, a3, p1, k1);
            store_inner(o1, base, s.v1);
            s.n0 = a2;
            s.n1 = a3;
            s.c0 = k1;
        }
        // march indices k = 1 .. L of U^{n+1} (index L is the far halo) and k-1 of U^{n+2}
        int k = 1;
        for (; k + G - 1 <= L; k += G) group<G, DIR>(s, base, k, L);
        for (; k <= L; ++k) group<1, DIR>(s, base, k, L);
    }
};

template <typename T, int VX, int G, bool C2F>
__global__ void __launch_bounds__(256) k_step2_march(StepArgs<T> p, T *__restrict__ u_next2, int cx0, int cx1,
                                                     int cy0, int cy1, int strips, int n_waves)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const int strip = w % strips, ty = w / strips;
    const int64_t boff = (int64_t)blockIdx.y * p.bstride;
    March2Ctx<T, VX, C2F> c;
    c.u = p.u + boff;
    c.up = p.uo + boff;
    c.c2 = C2F ? p.c2 : nullptr;
    c.o1 = p.uout + boff;
    c.o2 = u_next2 + boff;
    c.inv_h2 = p.inv_h2;
    c.dt2 = p.dt2;
    c.c2c = p.c2_const;
    c.nx = p.nx;
    c.ny = p.ny;
    c.cx0 = cx0;
    c.cx1 = cx1;
    c.cy0 = cy0;
    c.cy1 = cy1;
    c.xs = cx0 + (strip * 62 + lane - 1) * VX;
    c.need = c.xs < cx1 + VX;                                // lanes further right feed nobody
    c.xw = c.xs % c.nx;
    if (c.xw < 0) c.xw += c.nx;
    c.vec = c.xw % VX == 0 && c.xw + VX <= c.nx;
    c.out = lane >= 1 && lane <= 62 && c.xs < cx1;
    const int rows = p.tile_rows;
    const int ya = cy0 + ty * rows, yb = min(ya + rows, cy1);
    if (ty & 1)
        c.template march<G, -1>(yb - 1, yb - ya);
    else
        c.template march<G, 1>(ya, yb - ya);
}

// ---------------------------------------------------------------------------
// Frame steps as wave marches (the frames of a problem set; one grid's frame
// in spans of a few rows, as the tuner chooses).  On a periodic 2D grid
// everything outside a
// rectangle S is two wrapped rectangles: the rows outside S (every column)
// and S's rows on the columns outside S (one strip across the x wrap).  A
// span is 64 consecutive columns [xs, xe) of one of them and a chunk of its
// rows [ys, ye), both counted past the array end where they wrap.  One wave
// takes one span and marches down its rows keeping U^n of rows y-1, y, y+1
// in registers, the loads of G rows issued together; x neighbours come from
// the adjacent lanes (lane 0 and lane 63 read the column beyond the wave,
// the lane past the last column reads that column's right neighbour).
// Every cell takes cell_update with the layer loads hoisted.
// ---------------------------------------------------------------------------
struct Span2 {
    int32_t prob, xs, xe, ys, ye, pad0, pad1, pad2;
};

template <typename T, int G>
__device__ __forceinline__ void frame_march_wave(const StepArgs<T> &p, const Span2 &s)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny;
    const int x = s.xs + lane;
    const bool act = x < s.xe;
    const bool need = x <= s.xe;
    const int xc = x % nx;
    int xo = 0;
    bool edge = false;
    if (lane == 0) {
        xo = (s.xs + nx - 1) % nx;
        edge = act;
    } else if (lane == 63) {
        xo = (s.xs + 64) % nx;
        edge = act;
    }
    // rows ys-1 .. ye lie in [-1, 2 ny): one conditional wrap
    auto row_of = [&](int y) -> int { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };
    const T *u = p.u;
    T *out = p.uout ? p.uout : p.uo;
    auto ld = [&](int yr) -> T { return need ? u[(int64_t)yr * nx + xc] : T(0); };
    // the lane shifts run on the whole wave; only the span's own lanes update
    // (cell_update also stores the cell's Phi/Psi, and a lane past the span
    // may wrap onto a column another wave owns)
    auto cell = [&](int yr, T um, T uc, T up, T old, T ed) {
        T uxm = from_left(uc), uxp = from_right(uc);
        if (lane == 0) uxm = ed;
        if (lane == 63) uxp = ed;
        if (act) {
            const int64_t idx = (int64_t)yr * nx + xc;
            const T r = cell_update<T, 2, 7, true>(p, xc, yr, 0, idx, uc, uxm, uxp, um, up, T(0), T(0), old);
            out[idx] = r;
            if (p.hist) p.hist[idx] = r;
        }
    };
    T w[G + 2];                 // w[0] = row y-1, w[1] = row y, w[2 + g] = row y+1+g
    w[0] = ld(row_of(s.ys - 1));
    w[1] = ld(row_of(s.ys));
    int y = s.ys;
    for (; y + G <= s.ye; y += G) {
        T old[G], ed[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int yr = row_of(y + g);
            w[2 + g] = ld(row_of(y + g + 1));
            old[g] = act ? p.uo[(int64_t)yr * nx + xc] : T(0);
            ed[g] = edge ? u[(int64_t)yr * nx + xo] : T(0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) cell(row_of(y + g), w[g], w[g + 1], w[g + 2], old[g], ed[g]);
        w[0] = w[G];
        w[1] = w[G + 1];
    }
    for (; y < s.ye; ++y) {
        const int yr = row_of(y);
        w[2] = ld(row_of(y + 1));
        const T old = act ? p.uo[(int64_t)yr * nx + xc] : T(0);
        const T ed = edge ? u[(int64_t)yr * nx + xo] : T(0);
        cell(yr, w[0], w[1], w[2], old, ed);
        w[0] = w[1];
        w[1] = w[2];
    }
}

// A frame step of one grid (and its batch members) over a span list.
template <typename T, int G>
__global__ void __launch_bounds__(256) k_step_frame_march(StepArgs<T> p, const Span2 *__restrict__ spans, int n)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n) return;                                      // whole waves; no barriers below
    select_member(p, (int)blockIdx.y);
    frame_march_wave<T, G>(p, spans[w]);
}

// A frame step of many problems over one span list (span.prob selects the
// problem's step arguments).
template <typename T, int G>
__global__ void __launch_bounds__(256) k_multi_frame_march(const StepArgs<T> *__restrict__ probs,
                                                           const Span2 *__restrict__ spans, int n)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n) return;                                      // whole waves; no barriers below
    const Span2 s = spans[w];
    frame_march_wave<T, G>(probs[s.prob], s);
}

// Many problems, two- and three-step passes: the waves of every problem's
// core in one launch.  Each problem's descriptor holds its step arguments
// (U^n, U^{n-1}, U^{n+1} in u, uo, uout; the core rectangle in skip; tile
// rows in tile_rows) and its U^{n+2} (and U^{n+3}); the work list holds one
// (problem, strip, tile row) entry per wave.
template <typename T>
struct MultiCore {
    StepArgs<T> p;
    T *next2;
    T *next3;         // U^{n+3} (three-step passes)
    T *pen, *fin;     // U^{n+NL-1}, U^{n+NL} (passes of NL >= 4 levels)
};

template <typename T, int VX, int G>
__global__ void __launch_bounds__(256) k_multi_step2_march(const MultiCore<T> *__restrict__ cores,
                                                           const TileRef *__restrict__ waves, int n_waves)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const TileRef t = waves[w];
    const StepArgs<T> &p = cores[t.prob].p;
    March2Ctx<T, VX, false> c;
    c.u = p.u;
    c.up = p.uo;
    c.c2 = nullptr;
    c.o1 = p.uout;
    c.o2 = cores[t.prob].next2;
    c.inv_h2 = p.inv_h2;
    c.dt2 = p.dt2;
    c.c2c = p.c2_const;
    c.nx = p.nx;
    c.ny = p.ny;
    c.cx0 = p.skip[0];
    c.cx1 = p.skip[1];
    c.cy0 = p.skip[2];
    c.cy1 = p.skip[3];
    c.xs = c.cx0 + (t.tx * 62 + lane - 1) * VX;
    c.need = c.xs < c.cx1 + VX;
    c.xw = c.xs % c.nx;
    if (c.xw < 0) c.xw += c.nx;
    c.vec = c.xw % VX == 0 && c.xw + VX <= c.nx;
    c.out = lane >= 1 && lane <= 62 && c.xs < c.cx1;
    const int rows = p.tile_rows;
    const int ya = c.cy0 + t.ty * rows, yb = min(ya + rows, c.cy1);
    if (t.ty & 1)
        c.template march<G, -1>(yb - 1, yb - ya);
    else
        c.template march<G, 1>(ya, yb - ya);
}

// ---------------------------------------------------------------------------
// Three steps per launch, 2D periodic grids: the same marching scheme one
// level deeper.  For march index k a wave reads U^n(k+1) and U^{n-1}(k) and
// computes U^{n+1}(k), U^{n+2}(k-1) and U^{n+3}(k-2) from rows held in
// registers.  It writes U^{n+3} of its tile and U^{n+2} off the core's
// boundary ring; U^{n+1} stays in registers: 4 words per core cell per
// three steps instead of 6 for two two-step passes.  Each side of a strip
// carries HL = ceil(3/VX) halo lanes.  The frame's three ordinary steps run
// on a second stream meanwhile and reach two (first step) and one (second
// step) cells into the core, which is where they need U^{n+1} and U^{n+2}.
// ---------------------------------------------------------------------------
template <typename T, int VX, bool C2F>
struct March3Ctx : March2Ctx<T, VX, C2F> {
    using Base = March2Ctx<T, VX, C2F>;
    using R = Row<T, VX>;
    T *o3;                         // U^{n+3}

    // rolling state at march index k: U^n at k-1, k; U^{n+1} at k-2, k-1;
    // U^{n+2} at k-3, k-2; c^2 at k-2, k-1
    struct State {
        R n0, n1, a0, a1, b0, b1, c0, c1;
    };

    // one march index k with every level guarded (prologue and tail)
    template <int DIR>
    __device__ __forceinline__ void one(State &s, int base, int k, int L) const
    {
        const R nn = this->load(this->u, this->wrapy(base + DIR * (k + 1)));
        const R pm = this->load(this->up, this->wrapy(base + DIR * k));
        R cn{};
        if (C2F) cn = this->load(this->c2, this->wrapy(base + DIR * k));
        const R v1 = this->template lev<DIR>(s.n0, s.n1, nn, pm, cn);           // U^{n+1}(k)
        R v2{};
        if (k - 1 >= -1) {
            v2 = this->template lev<DIR>(s.a0, s.a1, v1, s.n0, s.c1);           // U^{n+2}(k-1)
            if (k - 1 >= 0 && k - 1 < L) this->store_inner(this->o2, base + DIR * (k - 1), v2);
        }
        if (k - 2 >= 0 && k - 2 < L)
            this->store(o3, base + DIR * (k - 2), this->template lev<DIR>(s.b0, s.b1, v2, s.a0, s.c0));
        s.n0 = s.n1;
        s.n1 = nn;
        s.a0 = s.a1;
        s.a1 = v1;
        s.b0 = s.b1;
        s.b1 = v2;
        s.c0 = s.c1;
        s.c1 = cn;
    }

    // G march indices k .. k+G-1 in the steady state (every level inside the
    // tile's range), all loads of the group issued first
    template <int G, int DIR>
    __device__ __forceinline__ void group(State &s, int base, int k) const
    {
        R wn[G + 2], pm[G], v1[G + 2], v2[G + 2], cw[G + 2];
        wn[0] = s.n0;
        wn[1] = s.n1;
        v1[0] = s.a0;
        v1[1] = s.a1;
        v2[0] = s.b0;
        v2[1] = s.b1;
        cw[0] = s.c0;
        cw[1] = s.c1;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            wn[2 + g] = this->load(this->u, this->wrapy(base + DIR * (k + 1 + g)));
            pm[g] = this->load(this->up, this->wrapy(base + DIR * (k + g)));
            if (C2F) cw[2 + g] = this->load(this->c2, this->wrapy(base + DIR * (k + g)));
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            v1[2 + g] = this->template lev<DIR>(wn[g], wn[g + 1], wn[g + 2], pm[g], cw[2 + g]);
            v2[2 + g] = this->template lev<DIR>(v1[g], v1[g + 1], v1[g + 2], wn[g], cw[g + 1]);
            this->store_inner(this->o2, base + DIR * (k - 1 + g), v2[2 + g]);
            this->store(o3, base + DIR * (k - 2 + g), this->template lev<DIR>(v2[g], v2[g + 1], v2[g + 2], v1[g], cw[g]));
        }
        s.n0 = wn[G];
        s.n1 = wn[G + 1];
        s.a0 = v1[G];
        s.a1 = v1[G + 1];
        s.b0 = v2[G];
        s.b1 = v2[G + 1];
        s.c0 = cw[G];
        s.c1 = cw[G + 1];
    }

    template <int G, int DIR>
    __device__ __forceinline__ void march(int base, int L) const
    {
        State s;
        s.n0 = this->load(this->u, this->wrapy(base - 3 * DIR));
        s.n1 = this->load(this->u, this->wrapy(base - 2 * DIR));
        s.a0 = s.a1 = s.b0 = s.b1 = s.c0 = s.c1 = R{};
        // march indices -2 .. 1: the levels fill up
        int k = -2;
        for (; k <= 1 && k <= L + 1; ++k) one<DIR>(s, base, k, L);
        // steady state: U^{n+1}(k) .. with k-2 >= 0 and k+G-1 <= L-1 (no guards needed)
        for (; k + G - 1 <= L - 1; k += G) group<G, DIR>(s, base, k);
        for (; k <= L + 1; ++k) one<DIR>(s, base, k, L);
    }
};

template <typename T, int VX, int G, bool C2F>
__global__ void __launch_bounds__(256) k_step3_march(StepArgs<T> p, T *__restrict__ u_next2, T *__restrict__ u_next3,
                                                     int cx0, int cx1, int cy0, int cy1, int strips, int n_waves)
{
    constexpr int HL = (3 + VX - 1) / VX;                    // halo lanes per side
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const int strip = w % strips, ty = w / strips;
    const int64_t boff = (int64_t)blockIdx.y * p.bstride;
    March3Ctx<T, VX, C2F> c;
    c.u = p.u + boff;
    c.up = p.uo + boff;
    c.c2 = C2F ? p.c2 : nullptr;
    c.o1 = p.uout + boff;
    c.o2 = u_next2 + boff;
    c.o3 = u_next3 + boff;
    c.inv_h2 = p.inv_h2;
    c.dt2 = p.dt2;
    c.c2c = p.c2_const;
    c.nx = p.nx;
    c.ny = p.ny;
    c.cx0 = cx0;
    c.cx1 = cx1;
    c.cy0 = cy0;
    c.cy1 = cy1;
    c.xs = cx0 + (strip * (64 - 2 * HL) + lane - HL) * VX;
    c.need = c.xs < cx1 + HL * VX;                           // lanes further right feed nobody
    c.xw = c.xs % c.nx;
    if (c.xw < 0) c.xw += c.nx;
    c.vec = c.xw % VX == 0 && c.xw + VX <= c.nx;
    c.out = lane >= HL && lane < 64 - HL && c.xs < cx1;
    const int rows = p.tile_rows;
    const int ya = cy0 + ty * rows, yb = min(ya + rows, cy1);
    if (ty & 1)
        c.template march<G, -1>(yb - 1, yb - ya);
    else
        c.template march<G, 1>(ya, yb - ya);
}

// ---------------------------------------------------------------------------
// NL steps per launch (NL >= 4), 2D grids: the marching scheme carried to any
// depth.  Level 0 is U^n, level l is U^{n+l}.  For march index k a wave reads
// U^n(k+1) and U^{n-1}(k) and forms level l on row k-l+1 (l = 1 .. NL) from
// level l-1 on rows k-l .. k-l+2 and level l-2 on row k-l+1, all held in
// registers.  It writes level NL on its tile and level NL-1 off the core's
// boundary ring; the levels below stay in registers (the frame's first steps
// write them where the later frame steps read them): 4 words per core cell
// per NL steps.  Level l is formed on rows [-(NL-l), L+NL-l) of a tile of L
// rows, so each side of a strip carries HL = ceil(NL/VX) halo lanes and a
// tile reads NL rows beyond each end.
// ---------------------------------------------------------------------------
// Point sources and receivers of a 2D pass (not part of the paper; the
// workload's shots and traces).  Level l of a pass from time index n is the
// step n+l-1: its sources add dt^2 w_s[n+l-1] / h^2 to U^{n+l} at their cells
// (every time a wave forms that cell at that level, halo copies included, so
// the levels built on it agree), and its receivers take U^{n+l} into trace
// column n+l-1.  The core records a receiver at level l when it lies at least
// NL-l cells inside the core (only the wave and lane that own the cell
// write); the frame's step l records the others from its own output.
template <typename T>
struct Taps2 {
    const int64_t *scells;     // source cells over the batch, ascending (member * cells + cell)
    const int64_t *sorder;     // caller's index of each sorted source
    const T *wav;              // wavelets [ns][nt_src]
    int32_t ns;                // sources (at most 32), 0: none
    int32_t nr;                // receivers, 0: none recorded
    int64_t nt_src, nt_rec;
    T amp;                     // dt^2 / h^2
    const int32_t *rmap;       // [member * ny + y]: first pool slot of row y's column map, or -1
    const int32_t *rpool;      // pool[slot + x]: receiver index of column x, or -1
    T *traces;                 // [nr][nt_rec]
    int64_t n;                 // time index of the pass's first step
};

template <typename T, int VX, bool C2F, int NL, bool HS = false>
struct MarchNCtx : March2Ctx<T, VX, C2F> {
    using R = Row<T, VX>;
    T *open, *ofin;                // U^{n+NL-1}, U^{n+NL}
    T *hist = nullptr;             // HS: U^{n+l} at hist + (l-1) * hstride for l < NL-1
    int64_t hstride = 0;
    Taps2<T> tp;                   // sources and receivers (tp.ns == 0 and tp.nr == 0: none)
    uint32_t smask = 0;            // sources this wave may form (bit q: the run starting at sorted q)
    int member = 0;
    bool taps = false;             // the tile has a source or receiver row: march with tap()

    // level l (1 .. NL) of this lane's cells on array row y: add the sources
    // there; record the receivers this lane owns (`own`: the row belongs to
    // the wave's tile)
    __device__ __forceinline__ void tap(R &v, int l, int y, bool own) const
    {
        const int nx = this->nx, ny = this->ny;
        const int64_t t = tp.n + l - 1;
        if (smask && t < tp.nt_src) {
            const int64_t mb = (int64_t)member * nx * ny;
            for (uint32_t m = smask; m; m &= m - 1) {
                const int q = __builtin_ctz(m);
                const int64_t cell = tp.scells[q] - mb;
                if ((int)(cell / nx) != y) continue;
                const int sx = (int)(cell % nx);
                T add = T(0);
                for (int r = q; r < tp.ns && tp.scells[r] == tp.scells[q]; ++r) add += tp.wav[tp.sorder[r] * tp.nt_src + t];
#pragma unroll
                for (int k = 0; k < VX; ++k) {
                    int x = (this->xs + k) % nx;
                    if (x < 0) x += nx;
                    if (x == sx) v.v[k] = v.v[k] + tp.amp * add;
                }
            }
        }
        if (tp.nr && own && this->out && t < tp.nt_rec) {
            const int slot = tp.rmap[(int64_t)member * ny + y];
            if (slot >= 0) {
#pragma unroll
                for (int k = 0; k < VX; ++k) {
                    const int x = this->xs + k;
                    if (x < this->cx0 || x >= this->cx1) continue;
                    const int ri = tp.rpool[slot + x];
                    const int d = min(min(x - this->cx0, this->cx1 - 1 - x), min(y - this->cy0, this->cy1 - 1 - y));
                    if (ri >= 0 && d >= NL - l) tp.traces[(int64_t)ri * tp.nt_rec + t] = v.v[k];
                }
            }
        }
    }

    // HS (history passes): level l < NL-1 of this lane's cells of row y at
    // depth >= NL-l inside the core; the frame's steps write the cells
    // nearer the core's edge, so every cell of level l has one writer
    __device__ __forceinline__ void store_level(int l, int y, const R &r) const
    {
        const int dd = NL - l;
        if (!this->out || y < this->cy0 + dd || y >= this->cy1 - dd) return;
        T *row = hist + (int64_t)(l - 1) * hstride + (int64_t)y * this->nx + this->xs;
        const int xa = this->cx0 + dd, xb = this->cx1 - dd;
        if (this->xs >= xa && this->xs + VX <= xb) {
            store_row<T, VX>(row, r);
        } else {
#pragma unroll
            for (int k = 0; k < VX; ++k)
                if (this->xs + k >= xa && this->xs + k < xb) row[k] = r.v[k];
        }
    }

    // rolling state at march index k: w[m] = level m on rows k-m-1, k-m
    // (m < NL); c[i] = c^2 on row k-NL+1+i (i < NL-1)
    struct State {
        R w[NL][2];
        R c[NL - 1];
    };

    // one march index k, every level guarded (prologue and tail; the whole
    // tile of a wave with sources or receivers, TAP)
    template <int DIR, bool TAP = false>
    __device__ __forceinline__ void one(State &s, int base, int k, int L) const
    {
        const R nn = this->load(this->u, this->wrapy(base + DIR * (k + 1)));
        const R pm = this->load(this->up, this->wrapy(base + DIR * k));
        R cn{};
        if (C2F) cn = this->load(this->c2, this->wrapy(base + DIR * k));
        advance<DIR, TAP>(s, base, k, L, nn, pm, cn);
    }

    // march index k from its loads: U^n(k+1), U^{n-1}(k), c^2(k); TAP: with
    // the sources and receivers of the level rows formed
    template <int DIR, bool TAP = false>
    __device__ __forceinline__ void advance(State &s, int base, int k, int L, const R &nn, const R &pm,
                                            const R &cn) const
    {
        R cur[NL + 1];                                  // level l formed on row k-l+1
        cur[0] = nn;
#pragma unroll
        for (int l = 1; l <= NL; ++l) {
            const int r = k - l + 1;
            cur[l] = R{};
            if (r < l - NL) continue;                   // below the rows level l is needed on
            const R &old = l == 1 ? pm : s.w[l >= 2 ? l - 2 : 0][0];
            const R &cl = l == 1 ? cn : s.c[l >= 2 ? NL - l : 0];
            cur[l] = this->template lev<DIR>(s.w[l - 1][0], s.w[l - 1][1], cur[l - 1], old, cl);
            if (TAP) tap(cur[l], l, this->wrapy(base + DIR * r), r >= 0 && r < L);
            if (HS && l < NL - 1 && r >= 0 && r < L) store_level(l, base + DIR * r, cur[l]);
            if (l == NL - 1 && r >= 0 && r < L) this->store_inner(open, base + DIR * r, cur[l]);
            if (l == NL && r >= 0 && r < L) this->store(ofin, base + DIR * r, cur[l]);
        }
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            s.w[m][0] = s.w[m][1];
            s.w[m][1] = cur[m];
        }
#pragma unroll
        for (int i = 0; i + 1 < NL - 1; ++i) s.c[i] = s.c[i + 1];
        s.c[NL - 2] = cn;
    }

    // the loads of the group at march index k: U^n rows k+1 .. k+G, U^{n-1}
    // and c^2 rows k .. k+G-1
    template <int G>
    struct Loads {
        R un[G], pm[G], c[G];
    };

    template <int G, int DIR>
    __device__ __forceinline__ void issue(Loads<G> &ld, int base, int k) const
    {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ld.un[g] = this->load(this->u, this->wrapy(base + DIR * (k + 1 + g)));
            ld.pm[g] = this->load(this->up, this->wrapy(base + DIR * (k + g)));
            if (C2F) ld.c[g] = this->load(this->c2, this->wrapy(base + DIR * (k + g)));
        }
    }

    // G march indices k .. k+G-1 in the steady state (every level's row inside
    // the tile), all loads of the group issued first
    template <int G, int DIR>
    __device__ __forceinline__ void group(State &s, int base, int k) const
    {
        Loads<G> ld;
        issue<G, DIR>(ld, base, k);
        compute<G, DIR>(s, base, k, ld);
    }

    template <int G, int DIR>
    __device__ __forceinline__ void compute(State &s, int base, int k, const Loads<G> &ld) const
    {
        R w[NL][G + 2], pm[G], cw[NL - 1 + G];         // w[m][i]: level m on row k-m-1+i
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            w[m][0] = s.w[m][0];
            w[m][1] = s.w[m][1];
        }
#pragma unroll
        for (int i = 0; i < NL - 1; ++i) cw[i] = s.c[i];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            w[0][2 + g] = ld.un[g];
            pm[g] = ld.pm[g];
            if (C2F) cw[NL - 1 + g] = ld.c[g];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int l = 1; l <= NL; ++l) {
                const R v = this->template lev<DIR>(w[l - 1][g], w[l - 1][g + 1], w[l - 1][g + 2],
                                                    l == 1 ? pm[g] : w[l >= 2 ? l - 2 : 0][g], cw[NL - l + g]);
                if (l < NL) w[l][2 + g] = v;
                if (HS && l < NL - 1) store_level(l, base + DIR * (k - l + 1 + g), v);
                if (l == NL - 1) this->store_inner(open, base + DIR * (k - l + 1 + g), v);
                if (l == NL) this->store(ofin, base + DIR * (k - l + 1 + g), v);
            }
        }
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            s.w[m][0] = w[m][G];
            s.w[m][1] = w[m][G + 1];
        }
#pragma unroll
        for (int i = 0; i < NL - 1; ++i) s.c[i] = cw[G + i];
    }

    // PF: every march index, prologue and tail included, takes loads issued
    // kAhead indices earlier (a ring of kAhead rows of each input in
    // registers) instead of the group scheme
    static constexpr int kAhead = 4;

    template <int G, int DIR, bool PF = false>
    __device__ __forceinline__ void march(int base, int L) const
    {
        State s;
#pragma unroll
        for (int m = 0; m < NL; ++m) s.w[m][0] = s.w[m][1] = R{};
#pragma unroll
        for (int i = 0; i < NL - 1; ++i) s.c[i] = R{};
        s.w[0][0] = this->load(this->u, this->wrapy(base - NL * DIR));
        s.w[0][1] = this->load(this->u, this->wrapy(base - (NL - 1) * DIR));
        int k = -(NL - 1);
        if (taps) {
            // a tile with sources or receivers: one march index at a time
            for (; k <= L + NL - 2; ++k) one<DIR, true>(s, base, k, L);
            return;
        }
        if (PF) {
            const int kend = L + NL - 2;
            R ru[kAhead], rp[kAhead], rc[kAhead];
#pragma unroll
            for (int q = 0; q < kAhead; ++q) {
                ru[q] = rp[q] = rc[q] = R{};
                if (k + q > kend) continue;
                ru[q] = this->load(this->u, this->wrapy(base + DIR * (k + q + 1)));
                rp[q] = this->load(this->up, this->wrapy(base + DIR * (k + q)));
                if (C2F) rc[q] = this->load(this->c2, this->wrapy(base + DIR * (k + q)));
            }
            for (; k <= kend; k += kAhead) {
#pragma unroll
                for (int q = 0; q < kAhead; ++q) {
                    const int kq = k + q;
                    if (kq > kend) break;
                    const R nn = ru[q], pm = rp[q], cn = rc[q];
                    if (kq + kAhead <= kend) {
                        ru[q] = this->load(this->u, this->wrapy(base + DIR * (kq + kAhead + 1)));
                        rp[q] = this->load(this->up, this->wrapy(base + DIR * (kq + kAhead)));
                        if (C2F) rc[q] = this->load(this->c2, this->wrapy(base + DIR * (kq + kAhead)));
                    }
                    advance<DIR>(s, base, kq, L, nn, pm, cn);
                }
            }
            return;
        }
        // march indices -(NL-1) .. NL-2: the levels fill up
        for (; k <= NL - 2 && k <= L + NL - 2; ++k) one<DIR>(s, base, k, L);
        // steady state: every level's rows inside the tile (no guards needed)
        for (; k + G - 1 <= L - 1; k += G) group<G, DIR>(s, base, k);
        for (; k <= L + NL - 2; ++k) one<DIR>(s, base, k, L);
    }
};

// Set up a march context for strip `strip`, tile row `ty` of the core
// [cx0, cx1) x [cy0, cy1) and run it.
template <typename T, int VX, int G, bool C2F, int NL, bool PF, bool HS = false>
__device__ __forceinline__ void run_marchN(const StepArgs<T> &p, const T *u, const T *uo, T *u_pen, T *u_fin,
                                           int cx0, int cx1, int cy0, int cy1, int strip, int ty, int lane,
                                           const Taps2<T> &tp = Taps2<T>{}, T *hist = nullptr,
                                           int64_t hstride = 0)
{
    constexpr int HL = (NL + VX - 1) / VX;                   // halo lanes per side
    MarchNCtx<T, VX, C2F, NL, HS> c;
    c.hist = hist;
    c.hstride = hstride;
    c.u = u;
    c.up = uo;
    c.c2 = C2F ? p.c2 : nullptr;
    c.o1 = nullptr;
    c.o2 = nullptr;
    c.open = u_pen;
    c.ofin = u_fin;
    c.inv_h2 = p.inv_h2;
    c.dt2 = p.dt2;
    c.c2c = p.c2_const;
    c.nx = p.nx;
    c.ny = p.ny;
    c.cx0 = cx0;
    c.cx1 = cx1;
    c.cy0 = cy0;
    c.cy1 = cy1;
    c.xs = cx0 + (strip * (64 - 2 * HL) + lane - HL) * VX;
    c.need = c.xs < cx1 + HL * VX;                           // lanes further right feed nobody
    c.xw = c.xs % c.nx;
    if (c.xw < 0) c.xw += c.nx;
    c.vec = c.xw % VX == 0 && c.xw + VX <= c.nx;
    c.out = lane >= HL && lane < 64 - HL && c.xs < cx1;
    const int rows = p.tile_rows;
    const int ya = cy0 + ty * rows, yb = min(ya + rows, cy1);
    c.tp = tp;
    c.member = (int)blockIdx.y;
    if (tp.ns > 0) {
        // the sources of this member whose row is within the rows the wave
        // forms at some level ([ya - NL, yb + NL)); columns are tested per lane
        const int64_t mb = (int64_t)c.member * p.nx * p.ny;
        for (int q = 0; q < tp.ns && q < 32; ++q) {
            const int64_t cell = tp.scells[q];
            if (q > 0 && tp.scells[q - 1] == cell) continue;
            if (cell < mb || cell >= mb + (int64_t)p.nx * p.ny) continue;
            const int sy = (int)((cell - mb) / p.nx);
            if (sy >= ya - NL && sy < yb + NL) c.smask |= 1u << q;
        }
    }
    c.taps = c.smask != 0;
    if (tp.nr > 0)
        for (int y = ya; y < yb && !c.taps; ++y) c.taps = tp.rmap[(int64_t)c.member * p.ny + y] >= 0;
    if (ty & 1)
        c.template march<G, -1, PF>(yb - 1, yb - ya);
    else
        c.template march<G, 1, PF>(ya, yb - ya);
}

template <typename T, int VX, int G, bool C2F, int NL, bool PF>
__global__ void __launch_bounds__(256) k_stepN_march(StepArgs<T> p, T *__restrict__ u_pen, T *__restrict__ u_fin,
                                                     int cx0, int cx1, int cy0, int cy1, int strips, int n_waves,
                                                     Taps2<T> tp)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int64_t boff = (int64_t)blockIdx.y * p.bstride;
    run_marchN<T, VX, G, C2F, NL, PF>(p, p.u + boff, p.uo + boff, u_pen + boff, u_fin + boff, cx0, cx1, cy0, cy1,
                                      w % strips, w / strips, (int)(threadIdx.x & 63), tp);
}

// The same pass storing every level (a history of U^{n+1} .. U^{n+NL} for
// the adjoint's recompute): levels below NL-1 go to hist + (l-1) * hstride
// on the core cells at depth >= NL-l, the last two to u_pen and u_fin as
// above.
template <typename T, int VX, int G, bool C2F, int NL>
__global__ void __launch_bounds__(256) k_stepN_hist(StepArgs<T> p, T *__restrict__ hist, int64_t hstride,
                                                    T *__restrict__ u_pen, T *__restrict__ u_fin, int cx0, int cx1,
                                                    int cy0, int cy1, int strips, int n_waves, Taps2<T> tp)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int64_t boff = (int64_t)blockIdx.y * p.bstride;
    run_marchN<T, VX, G, C2F, NL, false, true>(p, p.u + boff, p.uo + boff, u_pen + boff, u_fin + boff, cx0, cx1,
                                               cy0, cy1, w % strips, w / strips, (int)(threadIdx.x & 63), tp,
                                               hist + boff, hstride);
}

// Receivers from a list: traces[idx[i]][t] = U[cells[i]] for i < count (the
// receivers a frame step owns at its level).
template <typename T>
__global__ void __launch_bounds__(256) k_record_list(const T *__restrict__ u, const int64_t *__restrict__ cells,
                                                     const int32_t *__restrict__ idx, int64_t count,
                                                     T *__restrict__ traces, int64_t nt, int64_t t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    traces[(int64_t)idx[i] * nt + t] = u[cells[i]];
}

template <typename T, int VX, int G>
__global__ void __launch_bounds__(256) k_multi_step3_march(const MultiCore<T> *__restrict__ cores,
                                                           const TileRef *__restrict__ waves, int n_waves)
{
    constexpr int HL = (3 + VX - 1) / VX;                    // halo lanes per side
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const TileRef t = waves[w];
    const StepArgs<T> &p = cores[t.prob].p;
    March3Ctx<T, VX, false> c;
    c.u = p.u;
    c.up = p.uo;
    c.c2 = nullptr;
    c.o1 = p.uout;
    c.o2 = cores[t.prob].next2;
    c.o3 = cores[t.prob].next3;
    c.inv_h2 = p.inv_h2;
    c.dt2 = p.dt2;
    c.c2c = p.c2_const;
    c.nx = p.nx;
    c.ny = p.ny;
    c.cx0 = p.skip[0];
    c.cx1 = p.skip[1];
    c.cy0 = p.skip[2];
    c.cy1 = p.skip[3];
    c.xs = c.cx0 + (t.tx * (64 - 2 * HL) + lane - HL) * VX;
    c.need = c.xs < c.cx1 + HL * VX;
    c.xw = c.xs % c.nx;
    if (c.xw < 0) c.xw += c.nx;
    c.vec = c.xw % VX == 0 && c.xw + VX <= c.nx;
    c.out = lane >= HL && lane < 64 - HL && c.xs < c.cx1;
    const int rows = p.tile_rows;
    const int ya = c.cy0 + t.ty * rows, yb = min(ya + rows, c.cy1);
    if (t.ty & 1)
        c.template march<G, -1>(yb - 1, yb - ya);
    else
        c.template march<G, 1>(ya, yb - ya);
}

template <typename T, int VX, int G, int NL>
__global__ void __launch_bounds__(256) k_multi_stepN_march(const MultiCore<T> *__restrict__ cores,
                                                           const TileRef *__restrict__ waves, int n_waves)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const TileRef t = waves[w];
    const MultiCore<T> &mc = cores[t.prob];
    run_marchN<T, VX, G, false, NL, false>(mc.p, mc.p.u, mc.p.uo, mc.pen, mc.fin, mc.p.skip[0], mc.p.skip[1],
                                           mc.p.skip[2], mc.p.skip[3], t.tx, t.ty, (int)(threadIdx.x & 63));
}

// All D frame steps of a 2D pass in one launch (overlapped tiling).  Each
// block owns a TX x TY tile of the frame (tiles on a fixed grid, listed where
// they meet everything outside the core shrunk by one) and loads the tile
// with a halo of D cells into LDS: U^n, U^{n-1} and the four compact layer
// arrays (Phi_x, Psi_x, Phi_y, Psi_y) of the cells on their bands.  Step j
// updates the extended region shrunk by j cells, so after D steps the tile
// holds levels D-1 and D exactly; halo cells are recomputed by every tile
// that needs them.  U of level j overwrites level j-2 in place (a cell reads
// its own old value only); the layer arrays are updated through registers
// between two barriers (a cell reads its neighbours' old values).  The block
// writes U^{n+D-1} outside the core shrunk by one, U^{n+D} outside the core
// and the layer arrays of level n+D (to the aux buffer it did not read).
// Cells beyond a reflecting wall are ghosts holding 0.  Every cell is
// updated in cell_update's operation order.
template <typename T, int D, int TX, int TY>
__global__ void __launch_bounds__(256) k_frame_fused2d(StepArgs<T> p, T *__restrict__ u_pen, T *__restrict__ u_fin,
                                                       const TileRef *__restrict__ tiles, int ntiles)
{
    constexpr int W = TX + 2 * D, HH = TY + 2 * D, E = W * HH;
    constexpr int K = (E + 255) / 256;                       // extended cells per thread
    constexpr int MAXM = 255;                                // sigma slots kept in LDS per axis
    __shared__ T su[2][E];                                   // two U levels, alternating
    __shared__ T sx[2][E];                                   // Phi_x, Psi_x
    __shared__ T sy[2][E];                                   // Phi_y, Psi_y
    __shared__ T ssig[2][MAXM + 1];                          // sigma_x, sigma_y by band slot
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;                              // whole blocks, before any barrier
    select_member(p, (int)blockIdx.y);
    const int64_t boff = (int64_t)blockIdx.y * p.bstride;
    u_pen += boff;
    u_fin += boff;
    const TileRef t = tiles[tile];
    const int nx = p.nx, ny = p.ny;
    const int ox = t.tx * TX - D, oy = t.ty * TY - D;        // extended origin, unwrapped
    const Axis<T> &A0 = p.ax[0];
    const Axis<T> &A1 = p.ax[1];
    const int tid = (int)threadIdx.x;
    // (an axis without a layer has no sigma table: sig is null there)
    if (A0.M > 0)
        for (int k = tid; k <= A0.M && k <= MAXM; k += 256) ssig[0][k] = A0.sig[k];
    if (A1.M > 0)
        for (int k = tid; k <= A1.M && k <= MAXM; k += 256) ssig[1][k] = A1.sig[k];
    // grid coordinate of an extended coordinate, or -1 past a reflecting wall
    auto gco = [](int v, int n, int wall) {
        if (v >= 0 && v < n) return v;
        if (wall) return -1;
        const int m = v % n;
        return m < 0 ? m + n : m;
    };
    // per owned extended cell: grid coordinates (-1: ghost or past the end)
    int gxs[K], gys[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = tid + 256 * i;
        gxs[i] = gys[i] = -1;
        if (e >= E) continue;
        const int gx = gco(ox + e % W, nx, A0.wall), gy = gco(oy + e / W, ny, A1.wall);
        if (gx < 0 || gy < 0) continue;
        gxs[i] = gx;
        gys[i] = gy;
    }
    // load U^n, U^{n-1} and the layer arrays of the extended region
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = tid + 256 * i;
        if (e >= E) break;
        const int gx = gxs[i], gy = gys[i];
        T a = T(0), b = T(0), px = T(0), qx = T(0), py = T(0), qy = T(0);
        if (gx >= 0) {
            const int64_t idx = (int64_t)gy * nx + gx;
            a = p.u[idx];
            b = p.uo[idx];
            if (A0.M > 0) {
                const int j = band_coord(A0, gx);
                if (j <= A0.M) {
                    const int64_t c = layer_base<0>(A0.M, nx, ny, gx, gy, 0) + j;
                    if (j < A0.M) px = A0.phi[c];
                    if (j > 0) qx = A0.psi[c];
                }
            }
            if (A1.M > 0) {
                const int j = band_coord(A1, gy);
                if (j <= A1.M) {
                    const int64_t c = layer_base<1>(A1.M, nx, ny, gx, gy, 0) + (int64_t)j * nx;
                    if (j < A1.M) py = A1.phi[c];
                    if (j > 0) qy = A1.psi[c];
                }
            }
        }
        su[0][e] = a;
        su[1][e] = b;
        sx[0][e] = px;
        sx[1][e] = qx;
        sy[0][e] = py;
        sy[1][e] = qy;
    }
    __syncthreads();
    int cur = 0;                                             // su[cur]: level j-1; su[1-cur]: level j-2
    for (int lv = 1; lv <= D; ++lv) {
        T npx[K], nqx[K], npy[K], nqy[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = tid + 256 * i;
            npx[i] = nqx[i] = npy[i] = nqy[i] = T(0);
            const int gx = gxs[i], gy = gys[i];
            if (gx < 0) continue;                            // ghosts stay 0
            const int ex = e % W, ey = e / W;
            if (ex < lv || ex >= W - lv || ey < lv || ey >= HH - lv) continue;
            const T *uc_ = su[cur];
            const T uc = uc_[e], uxm = uc_[e - 1], uxp = uc_[e + 1], uym = uc_[e - W], uyp = uc_[e + W];
            const T uold = su[1 - cur][e];
            T lap = ((uxm - T(2) * uc) + uxp) * p.inv_h2;
            lap += ((uym - T(2) * uc) + uyp) * p.inv_h2;
            const T c2 = p.c2 ? p.c2[(int64_t)gy * nx + gx] : p.c2_const;
            T damp = T(0);
            if (A0.M > 0) {
                const int j = band_coord(A0, gx);
                if (j <= A0.M) {
                    const bool lg = A0.wall && j == A0.hi, rg = A0.wall && j == A0.hi - 1;
                    const T s = j <= MAXM ? ssig[0][j] : A0.sig[j];
                    const T sl = (j > 0 && !lg) ? (j - 1 <= MAXM ? ssig[0][j - 1] : A0.sig[j - 1]) : T(0);
                    const T phi_l = (j > 0 && !lg) ? sx[0][e - 1] : T(0);
                    const T psi_r = (j < A0.M && !rg) ? sx[1][e + 1] : T(0);
                    const T grad = (uxp - uxm) * p.inv_2h;
                    if (j < A0.M) {
                        const T phi_c = sx[0][e];
                        npx[i] = phi_c + p.dt * (T(-0.5) * (sl * phi_l + s * phi_c) - grad);
                    }
                    if (j > 0) {
                        const T psi_c = sx[1][e];
                        nqx[i] = psi_c + p.dt * (T(-0.5) * (sl * psi_c + s * psi_r) - grad);
                    }
                    damp += (s * psi_r - sl * phi_l) * p.inv_h;
                }
            }
            if (A1.M > 0) {
                const int j = band_coord(A1, gy);
                if (j <= A1.M) {
                    const bool lg = A1.wall && j == A1.hi, rg = A1.wall && j == A1.hi - 1;
                    const T s = j <= MAXM ? ssig[1][j] : A1.sig[j];
                    const T sl = (j > 0 && !lg) ? (j - 1 <= MAXM ? ssig[1][j - 1] : A1.sig[j - 1]) : T(0);
                    const T phi_l = (j > 0 && !lg) ? sy[0][e - W] : T(0);
                    const T psi_r = (j < A1.M && !rg) ? sy[1][e + W] : T(0);
                    const T grad = (uyp - uym) * p.inv_2h;
                    if (j < A1.M) {
                        const T phi_c = sy[0][e];
                        npy[i] = phi_c + p.dt * (T(-0.5) * (sl * phi_l + s * phi_c) - grad);
                    }
                    if (j > 0) {
                        const T psi_c = sy[1][e];
                        nqy[i] = psi_c + p.dt * (T(-0.5) * (sl * psi_c + s * psi_r) - grad);
                    }
                    damp += (s * psi_r - sl * phi_l) * p.inv_h;
                }
            }
            const T rhs = c2 * lap + damp;
            su[1 - cur][e] = (T(2) * uc - uold) + p.dt2 * rhs;
        }
        __syncthreads();                                     // every old layer value has been read
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = tid + 256 * i;
            const int gx = gxs[i], gy = gys[i];
            if (gx < 0) continue;
            const int ex = e % W, ey = e / W;
            if (ex < lv || ex >= W - lv || ey < lv || ey >= HH - lv) continue;
            if (A0.M > 0) {
                const int j = band_coord(A0, gx);
                if (j <= A0.M) {
                    if (j < A0.M) sx[0][e] = npx[i];
                    if (j > 0) sx[1][e] = nqx[i];
                }
            }
            if (A1.M > 0) {
                const int j = band_coord(A1, gy);
                if (j <= A1.M) {
                    if (j < A1.M) sy[0][e] = npy[i];
                    if (j > 0) sy[1][e] = nqy[i];
                }
            }
        }
        __syncthreads();
        cur = 1 - cur;
    }
    // the tile's own cells: su[cur] = level D, su[1-cur] = level D-1
    for (int e2 = tid; e2 < TX * TY; e2 += 256) {
        const int tx = e2 % TX, ty = e2 / TX;
        const int gx = t.tx * TX + tx, gy = t.ty * TY + ty;
        if (gx >= nx || gy >= ny) continue;
        const int e = (ty + D) * W + tx + D;
        const int64_t idx = (int64_t)gy * nx + gx;
        const bool core0 = gx >= p.skip[0] && gx < p.skip[1] && gy >= p.skip[2] && gy < p.skip[3];
        const bool core1 = gx > p.skip[0] && gx < p.skip[1] - 1 && gy > p.skip[2] && gy < p.skip[3] - 1;
        if (!core0) u_fin[idx] = su[cur][e];
        if (!core1) u_pen[idx] = su[1 - cur][e];
        if (A0.M > 0) {
            const int j = band_coord(A0, gx);
            if (j <= A0.M) {
                const int64_t c = layer_base<0>(A0.M, nx, ny, gx, gy, 0) + j;
                if (j < A0.M) A0.phi_o[c] = sx[0][e];
                if (j > 0) A0.psi_o[c] = sx[1][e];
            }
        }
        if (A1.M > 0) {
            const int j = band_coord(A1, gy);
            if (j <= A1.M) {
                const int64_t c = layer_base<1>(A1.M, nx, ny, gx, gy, 0) + (int64_t)j * nx;
                if (j < A1.M) A1.phi_o[c] = sy[0][e];
                if (j > 0) A1.psi_o[c] = sy[1][e];
            }
        }
    }
}

// One ordinary step over a list of 64 x 4 cell tiles (the frame around the
// core), leaving the core cells (p.skip) alone.
template <typename T>
__global__ void __launch_bounds__(256) k_step_frame(StepArgs<T> p, const TileRef *__restrict__ tiles, int ntiles)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    select_member(p, (int)blockIdx.y);
    const TileRef t = tiles[tile];
    const int x = t.tx * 64 + (int)(threadIdx.x % 64);
    const int y = t.ty * 4 + (int)(threadIdx.x / 64);
    if (x >= p.skip[0] && x < p.skip[1] && y >= p.skip[2] && y < p.skip[3]) return;
    cell2d_tile<T, 4>(p, t.tx, t.ty);
}

// ---------------------------------------------------------------------------
// Many independent 2D problems of different sizes in one launch: a flat
// work list of tiles (problem, tile column, tile row) over all problems; each
// block looks up its problem's arguments (uniform, read through the scalar
// cache) and runs one marching tile.
// ---------------------------------------------------------------------------
// Many problems: each block takes one tile of (256 VX) columns x tile_rows
// rows of one problem from the work list and marches down it (the shape the
// tuner prefers for single 2D grids), so the per-block lookup of the
// problem's arguments is amortised over 1024 VX cells.
template <typename T, int VX, int R>
__global__ void __launch_bounds__(256) k_step_multi2d(const StepArgs<T> *__restrict__ probs,
                                                      const TileRef *__restrict__ tiles, int ntiles)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const TileRef t = tiles[tile];
    const StepArgs<T> p = probs[t.prob];
    // pad != 0: the tile holds cells with damping terms (layer code, hoisted
    // loads); otherwise the plain stencil
    if (t.pad)
        march2d_tile<T, VX, R, true>(p, t.tx, t.ty);
    else
        march2d_tile<T, VX, R, false, 0>(p, t.tx, t.ty);
}

// ---------------------------------------------------------------------------
// Variant MARCH, 3D: each wave owns 64 consecutive columns x RY rows of an
// (x, y) plane and marches through `tile_rows` planes in z, keeping U^n of
// planes z-1, z, z+1 for its RY rows in registers, so every plane of U^n is
// read once per chunk.  x neighbours come from the adjacent lanes (cross-lane
// shuffles; lanes 0 and 63 read the one column beyond the strip), y
// neighbours from the adjacent register rows (the rows just above and below
// the wave come from the L2 cache, where the neighbouring waves read them as
// their own).  A block's 4 waves take 4 consecutive row groups.
//
// The kernel updates the cells of one box: columns [xs, xe), rows [ys, ye)
// and planes [zs, ze), each start inside the array and each extent at most
// the axis length; indices past the array end continue at its start.  That
// wrap is the periodic one, so the two halves of a layer band are one box;
// with reflecting walls the neighbours across a wall read zero instead.
// AX is the set of axes whose layer terms the box's cells may meet: none on
// the layer-free core, x on the x-band strip (its layer inputs fetched one
// plane ahead).  The library splits a step into such boxes so that each
// kernel keeps only the code its cells need.
// ---------------------------------------------------------------------------
struct Box3 {
    int32_t xs, xe, ys, ye, zs, ze;
};

template <typename T, int RY, int AX>
__global__ void __launch_bounds__(256) k_step_zmarch3d(StepArgs<T> p, Box3 bx)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
    select_member(p, (int)blockIdx.y);
    const int per_plane = p.tiles_x * p.tiles_y;
    const int tz = tile / per_plane;
    const int rem = tile - tz * per_plane;
    const int ty = rem / p.tiles_x;
    const int tx = rem - ty * p.tiles_x;
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int y0 = bx.ys + (ty * 4 + (int)(threadIdx.x >> 6)) * RY;
    if (y0 >= bx.ye) return;                               // whole wave; no barriers below
    const bool wx = p.ax[0].wall, wy = p.ax[1].wall, wz = p.ax[2].wall;
    const int64_t sxy = (int64_t)nx * ny;
    // lane column x (unwrapped) and the array column it reads; the lane just
    // past the box's last column still reads, as that column's neighbour
    const int x0 = bx.xs + tx * 64, x = x0 + lane;
    const bool act = x < bx.xe;
    const bool need = x <= bx.xe;
    const int xc = x % nx;
    // lanes 0 and 63 also read the column just outside the strip
    int xo = 0;
    if (lane == 0) xo = x0 == 0 ? nx - 1 : (x0 - 1) % nx;
    else if (lane == 63) xo = (x0 + 64) % nx;
    const bool edge = (lane == 0 || lane == 63) && act;
    // walls: neighbours across the wall are zero (the ghost cells)
    const bool x_lo_wall = wx && xc == 0, x_hi_wall = wx && xc == nx - 1;
    // register rows q = 0..RY-1 and the halo rows above and below, as array rows
    int ry[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) ry[q] = (y0 + q) % ny;
    const int rlo = y0 == 0 ? ny - 1 : (y0 - 1) % ny, rhi = (y0 + RY) % ny;
    const T *u = p.u;
    auto ld = [&](int pz, int r) -> T { return need ? u[(int64_t)pz * sxy + (int64_t)r * nx + xc] : T(0); };
    const int z0 = bx.zs + tz * p.tile_rows;
    const int z1 = min(z0 + p.tile_rows, bx.ze);
    T um[RY], uc[RY];
    {
        const int zc = z0 % nz, pm = zc == 0 ? nz - 1 : zc - 1;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            um[q] = ld(pm, ry[q]);
            uc[q] = ld(zc, ry[q]);
        }
    }
    T *out = p.uout ? p.uout : p.uo;
    // the loads plane z needs beyond the window: U^n of plane z+1, U^{n-1}
    // of plane z, the strip-edge columns and the halo rows of plane z.  They
    // are issued one plane ahead, so a wave computes plane z while the
    // loads of plane z+1 are in flight.
    // With the x-layer terms alone (AX = 1) the layer inputs of the plane
    // (Phi_x, Psi_x around the cell's band slot) are fetched one plane ahead too.
    struct Fetch {
        T upn[RY], old[RY], edge[RY], hlo, hhi;
        LayerIn<T> lx[AX == 1 ? RY : 1];
    };
    const int jx = (AX == 1 && p.ax[0].M > 0 && act) ? band_coord(p.ax[0], xc) : (1 << 30);
    auto fetch = [&](int z, Fetch &f) {
        const int zc = z % nz;
        const int pz = zc == nz - 1 ? 0 : zc + 1;
        const int64_t plane = (int64_t)zc * sxy;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const bool row = y0 + q < bx.ye;
            f.upn[q] = ld(pz, ry[q]);
            f.old[q] = (act && row) ? p.uo[plane + (int64_t)ry[q] * nx + xc] : T(0);
            f.edge[q] = (edge && row) ? u[plane + (int64_t)ry[q] * nx + xo] : T(0);
            if constexpr (AX == 1) {
                f.lx[q].on = false;
                if (row && jx <= p.ax[0].M) f.lx[q] = layer_load<0>(p.ax[0], jx, nx, ny, xc, ry[q], zc);
            }
        }
        f.hlo = ld(zc, rlo);
        f.hhi = ld(zc, rhi);
    };
    Fetch cur;
    if (z0 < z1) fetch(z0, cur);
    for (int z = z0; z < z1; ++z) {
        Fetch nxt;
        if (z + 1 < z1) fetch(z + 1, nxt);
        const int zc = z % nz;
        const int64_t plane = (int64_t)zc * sxy;
        const bool z_lo_wall = wz && zc == 0, z_hi_wall = wz && zc == nz - 1;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            T uxm = __shfl_up(uc[q], 1);
            T uxp = __shfl_down(uc[q], 1);
            if (lane == 0) uxm = cur.edge[q];
            if (lane == 63) uxp = cur.edge[q];
            if (x_lo_wall) uxm = T(0);
            if (x_hi_wall) uxp = T(0);
            T uym = q == 0 ? cur.hlo : uc[q - 1];
            T uyp = q == RY - 1 ? cur.hhi : uc[q + 1];
            if (wy && ry[q] == 0) uym = T(0);
            if (wy && ry[q] == ny - 1) uyp = T(0);
            const T uzm = z_lo_wall ? T(0) : um[q];
            const T uzp = z_hi_wall ? T(0) : cur.upn[q];
            if (act && y0 + q < bx.ye) {
                const int64_t idx = plane + (int64_t)ry[q] * nx + xc;
                T r;
                if constexpr (AX == 1) {
                    // cell_update's hoisted form with the prefetched x-layer inputs
                    const T c2 = p.c2 ? p.c2[idx] : p.c2_const;
                    T lap = ((uxm - T(2) * uc[q]) + uxp) * p.inv_h2;
                    lap += ((uym - T(2) * uc[q]) + uyp) * p.inv_h2;
                    lap += ((uzm - T(2) * uc[q]) + uzp) * p.inv_h2;
                    T damp = T(0);
                    if (cur.lx[q].on) damp += layer_finish(p.ax[0], cur.lx[q], jx, uxm, uxp, p.dt, p.inv_2h) * p.inv_h;
                    const T rhs = c2 * lap + damp;
                    r = (T(2) * uc[q] - cur.old[q]) + p.dt2 * rhs;
                } else {
                    r = cell_update<T, 3, AX, (AX != 0)>(p, xc, ry[q], zc, idx, uc[q], uxm, uxp, uym, uyp, uzm,
                                                         uzp, cur.old[q]);
                }
                out[idx] = r;
                if (p.hist) p.hist[idx] = r;
            }
        }
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            um[q] = uc[q];
            uc[q] = cur.upn[q];
        }
        cur = nxt;
    }
}

// The same box update one thread per cell (64 x 4 cells of a plane per
// block): for boxes whose cells mostly carry layer terms, where many waves in
// flight hide the latency of the layer loads better than a plane march.
// Consecutive tiles take the same (x, y) tile on up to 8 consecutive planes,
// then the next (x, y) tile: the planes above and below a tile are read by
// its neighbours in launch order (L2 hits), and the tiles sharing its halo
// rows are at most 8 tiles-per-row further on.
template <typename T, int AX>
__global__ void __launch_bounds__(256) k_step_box3d(StepArgs<T> p, Box3 bx)
{
    constexpr int ZG = 8;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
    select_member(p, (int)blockIdx.y);
    const int per_plane = p.tiles_x * p.tiles_y;
    const int g = tile / (per_plane * ZG);                 // group of ZG planes
    const int zn = min(ZG, bx.ze - bx.zs - g * ZG);        // planes in this group
    const int rem = tile - g * per_plane * ZG;
    const int xy = rem / zn;
    const int tz = g * ZG + (rem - xy * zn);
    const int ty = xy / p.tiles_x;
    const int tx = xy - ty * p.tiles_x;
    const int xu = bx.xs + tx * 64 + (int)(threadIdx.x & 63);
    const int yu = bx.ys + ty * 4 + (int)(threadIdx.x >> 6);
    if (xu >= bx.xe || yu >= bx.ye) return;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    // box starts lie in the array and extents are at most its length: one wrap
    const int zu = bx.zs + tz;
    const int x = xu >= nx ? xu - nx : xu, y = yu >= ny ? yu - ny : yu, z = zu >= nz ? zu - nz : zu;
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t plane = (int64_t)z * sxy;
    const int64_t row = plane + (int64_t)y * nx;
    const int64_t idx = row + x;
    const T *u = p.u;
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    const int zm = wrap_dec(z, nz), zp = wrap_inc(z, nz);
    const T uzm = (p.ax[2].wall && z == 0) ? T(0) : u[(int64_t)zm * sxy + (int64_t)y * nx + x];
    const T uzp = (p.ax[2].wall && z == nz - 1) ? T(0) : u[(int64_t)zp * sxy + (int64_t)y * nx + x];
    const T uxm = (p.ax[0].wall && x == 0) ? T(0) : u[row + xm];
    const T uxp = (p.ax[0].wall && x == nx - 1) ? T(0) : u[row + xp];
    const T uym = (p.ax[1].wall && y == 0) ? T(0) : u[plane + (int64_t)ym * nx + x];
    const T uyp = (p.ax[1].wall && y == ny - 1) ? T(0) : u[plane + (int64_t)yp * nx + x];
    const T r = cell_update<T, 3, AX, true>(p, x, y, z, idx, u[idx], uxm, uxp, uym, uyp, uzm, uzp, p.uo[idx]);
    (p.uout ? p.uout : p.uo)[idx] = r;
    if (p.hist) p.hist[idx] = r;
}

// ---------------------------------------------------------------------------
// Variant TWOSTEP, 3D: two steps per pass over the core box, where no damping
// term acts within two cells.  A wave holds 64 consecutive columns (the two
// outer lanes on each side are halo) x RY rows and marches through a chunk of
// planes.  At march plane k it forms U^{n+1} on plane k for the rows
// -1 .. RY (from U^n of planes k-1, k, k+1 and U^{n-1} of plane k), then
// U^{n+2} on plane k-1 for the rows 0 .. RY-1 from the U^{n+1} planes k-2,
// k-1, k, all held in registers: per cell it reads U^n and U^{n-1} and
// writes U^{n+1} (on the inner box only: the frame's own steps write the
// ring around it) and U^{n+2}.  Both levels evaluate cell_update's
// expressions in its order with no damping terms, so the results are
// bit-identical to single steps.  Point sources within the wave's reach are
// added to both levels as the single steps add them.
// ---------------------------------------------------------------------------
template <typename T>
struct Src3 {
    const int64_t *cells;   // source cells in ascending order
    const int64_t *order;   // caller's index of each sorted source
    const T *wav;           // wavelets [ns][nt]
    int64_t ns, nt;
    int64_t n;              // time index of the first level
    T amp;                  // dt^2 / h^3
};

// d = (s - start) mod n in [0, n): is s within `len` cells from start?
__device__ __forceinline__ bool in_window(int s, int start, int len, int n)
{
    int d = (s - start) % n;
    if (d < 0) d += n;
    return len >= n || d < len;
}

// ORD = 1 takes tiles in launch order (the XCDs interleaved, so the whole
// GPU marches through the same chunk of planes at a time); ORD = 0 gives
// each XCD a consecutive run of tiles.
template <typename T, int RY, int ORD = 0>
__global__ void __launch_bounds__(256) k_step2_zmarch3d(StepArgs<T> p, T *__restrict__ u_next2, Box3 c, Box3 in1,
                                                        Src3<T> src)
{
    constexpr int NR = RY + 2;                               // rows of the first level: -1 .. RY
    const int tile = ORD ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= p.n_tiles) return;
    const int per_plane = p.tiles_x * p.tiles_y;
    const int tz = tile / per_plane;
    const int rem = tile - tz * per_plane;
    const int ty = rem / p.tiles_x;
    const int tx = rem - ty * p.tiles_x;
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int y0 = c.ys + (ty * 4 + wv) * RY;                 // first output row (unwrapped)
    if (y0 >= c.ye) return;                                   // whole wave; no barriers below
    const int64_t sxy = (int64_t)nx * ny;
    const int xw0 = c.xs - 2 + tx * 60;                       // the wave's first column (unwrapped)
    const int xu = xw0 + lane;
    const int xc = ((xu % nx) + nx) % nx;
    const bool xout = lane >= 2 && lane < 62 && xu < c.xe;   // U^{n+2} column
    const bool xin1 = xout && xu >= in1.xs && xu < in1.xe;   // U^{n+1} stored too
    const bool need = xu < c.xe + 2;                          // lanes past the reach read nothing
    // array rows of the relative rows -2 .. RY+1
    int ra[RY + 4];
#pragma unroll
    for (int r = 0; r < RY + 4; ++r) ra[r] = (((y0 - 2 + r) % ny) + ny) % ny;
    const int z0 = c.zs + tz * p.tile_rows;
    const int z1 = min(z0 + p.tile_rows, c.ze);
    // planes z0-2 .. z1+1 lie in [-2, 2 nz): one conditional wrap
    auto zwrap = [&](int z) -> int { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
    const T *u = p.u;
    // a row's base is the same for the whole wave, the lane adds its column
    const uint32_t xo = (uint32_t)xc;
    // per-lane byte offsets of the relative rows -2 .. RY+1 within a plane
    // (a plane is below 4 GiB): every access is a plane's base, one scalar
    // pair per plane and array, plus one of these 32-bit offsets
    uint32_t ob[RY + 4];
#pragma unroll
    for (int r = 0; r < RY + 4; ++r) ob[r] = ((uint32_t)ra[r] * (uint32_t)nx + xo) * (uint32_t)sizeof(T);
    auto pbase = [&](const T *b, int zc) -> const char * {
        const uint64_t v = (uint64_t)(b + (int64_t)zc * sxy);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
        return (const char *)(((uint64_t)hi << 32) | lo);
    };
    auto ld = [&](const char *pb, int r) -> T { return need ? *(const T *)(pb + ob[r]) : T(0); };
    // sources whose cell lies in the wave's reach (first level: rows -1..RY,
    // planes z0-1 .. z1): bit q for the run of equal cells starting at q
    uint32_t smask = 0;
    for (int q = 0; q < (int)src.ns && q < 32; ++q) {
        const int64_t cell = src.cells[q];
        if (q > 0 && src.cells[q - 1] == cell) continue;
        const int sz = (int)(cell / sxy), sy = (int)((cell / nx) % ny), sx = (int)(cell % nx);
        if (in_window(sx, xw0, 64, nx) && in_window(sy, y0 - 1, NR, ny) && in_window(sz, z0 - 1, z1 - z0 + 2, nz))
            smask |= 1u << q;
    }
    // add the sources on plane zc at time index tn to the rows of v (relative rows r0 ..)
    auto inject = [&](auto &v, int r0, int zc, int64_t tn) {
        constexpr int NV = (int)(sizeof(v) / sizeof(v[0]));
        if (tn >= src.nt) return;
        for (uint32_t m = smask; m; m &= m - 1) {
            const int q = __builtin_ctz(m);
            const int64_t cell = src.cells[q];
            if ((int)(cell / sxy) != zc) continue;
            const int sy = (int)((cell / nx) % ny), sx = (int)(cell % nx);
            T add = T(0);
            for (int64_t r = q; r < src.ns && src.cells[r] == cell; ++r) add += src.wav[src.order[r] * src.nt + tn];
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if ((((y0 + r0 + i) % ny) + ny) % ny == sy && xc == sx) v[i] = v[i] + src.amp * add;
        }
    };
    // one step of a cell in cell_update's order (c^2 constant, no damping terms)
    const T inv_h2 = p.inv_h2, dt2 = p.dt2, c2c = p.c2_const;
    auto upd = [&](T uc, T uxm, T uxp, T uym, T uyp, T uzm, T uzp, T old) -> T {
        T lap = ((uxm - T(2) * uc) + uxp) * inv_h2;
        lap += ((uym - T(2) * uc) + uyp) * inv_h2;
        lap += ((uzm - T(2) * uc) + uzp) * inv_h2;
        const T rhs = c2c * lap + T(0);
        return (T(2) * uc - old) + dt2 * rhs;
    };
    // U^n of planes k-1, k, k+1 (rows -1 .. RY); U^{n+1} of planes k-2 (rows
    // 0 .. RY-1), k-1 and k (rows -1 .. RY)
    T n0[NR], n1[NR], a0[RY], a1[NR];
    struct Fetch {
        T n2[NR], old[NR], hlo, hhi;
    };
    auto fetch = [&](int k, Fetch &f) {
        const int zc = zwrap(k), zn = zwrap(k + 1);
        const char *un = pbase(u, zn), *uc = pbase(u, zc), *uoc = pbase(p.uo, zc);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            f.n2[i] = ld(un, i + 1);
            f.old[i] = ld(uoc, i + 1);
        }
        f.hlo = ld(uc, 0);
        f.hhi = ld(uc, RY + 3);
    };
    {
        const char *um = pbase(u, zwrap(z0 - 2)), *uc = pbase(u, zwrap(z0 - 1));
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            n0[i] = ld(um, i + 1);
            n1[i] = ld(uc, i + 1);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) a1[i] = T(0);
#pragma unroll
    for (int i = 0; i < RY; ++i) a0[i] = T(0);
    T *out1 = p.uout;
    Fetch cur;
    fetch(z0 - 1, cur);
    for (int k = z0 - 1; k <= z1; ++k) {
        Fetch nxt;
        if (k + 1 <= z1) fetch(k + 1, nxt);
        const int zc = zwrap(k);
        // level 1: U^{n+1} on plane k, rows -1 .. RY
        T a2[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const T uc = n1[i];
            const T uxm = from_left(uc), uxp = from_right(uc);
            const T uym = i == 0 ? cur.hlo : n1[i - 1];
            const T uyp = i == NR - 1 ? cur.hhi : n1[i + 1];
            a2[i] = upd(uc, uxm, uxp, uym, uyp, n0[i], cur.n2[i], cur.old[i]);
        }
        if (smask) inject(a2, -1, zc, src.n);
        if (k >= z0 && k < z1 && k >= in1.zs && k < in1.ze) {
            char *ob1 = (char *)pbase(out1, zc);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int y = y0 + r;
                if (xin1 && y < c.ye && y >= in1.ys && y < in1.ye) *(T *)(ob1 + ob[r + 2]) = a2[r + 1];
            }
        }
        // level 2: U^{n+2} on plane k-1, rows 0 .. RY-1
        if (k >= z0 + 1) {
            const int zp = zwrap(k - 1);
            T v[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const T uc = a1[r + 1];
                const T uxm = from_left(uc), uxp = from_right(uc);
                v[r] = upd(uc, uxm, uxp, a1[r], a1[r + 2], a0[r], a2[r + 1], n0[r + 1]);
            }
            if (smask) inject(v, 0, zp, src.n + 1);
            char *ob2 = (char *)pbase(u_next2, zp);
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (xout && y0 + r < c.ye) *(T *)(ob2 + ob[r + 2]) = v[r];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) a0[r] = a1[r + 1];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            a1[i] = a2[i];
            n0[i] = n1[i];
            n1[i] = cur.n2[i];
        }
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// Start: U^{-1} = U^0 - dt V^0 + dt^2/2 c^2 Lap(U^0)  (Phi = Psi = 0).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_start(const T *__restrict__ u0, const T *__restrict__ v0,
                                               T *__restrict__ um1, const T *__restrict__ c2,
                                               T c2_const, T inv_h2, T dt, T half_dt2,
                                               int nx, int ny, int nz, int walls)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = D == 3 ? (int)(blockIdx.z % nz) : 0;
    const int bi = D == 3 ? (int)(blockIdx.z / nz) : (int)blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t boff = (int64_t)bi * nx * ny * nz;
    u0 += boff;
    um1 += boff;
    if (v0) v0 += boff;
    const int64_t sx = nx, sxy = (int64_t)nx * ny;
    const int64_t idx = (int64_t)z * sxy + (int64_t)y * sx + x;
    const int64_t plane = (int64_t)z * sxy;
    const T c = u0[idx];
    // neighbour values (0 on ghost cells past a wall; bit a of `walls` set for axis a)
    const bool wx = walls & 1, wy = walls & 2, wz = walls & 4;
    const T xm_ = (wx && x == 0) ? T(0) : u0[plane + (int64_t)y * sx + wrap_dec(x, nx)];
    const T xp_ = (wx && x == nx - 1) ? T(0) : u0[plane + (int64_t)y * sx + wrap_inc(x, nx)];
    const T ym_ = (wy && y == 0) ? T(0) : u0[plane + (int64_t)wrap_dec(y, ny) * sx + x];
    const T yp_ = (wy && y == ny - 1) ? T(0) : u0[plane + (int64_t)wrap_inc(y, ny) * sx + x];
    T lap = T(0);
    lap += ((xm_ - T(2) * c) + xp_) * inv_h2;
    lap += ((ym_ - T(2) * c) + yp_) * inv_h2;
    if (D == 3) {
        const T zm_ = (wz && z == 0) ? T(0) : u0[(int64_t)wrap_dec(z, nz) * sxy + (int64_t)y * sx + x];
        const T zp_ = (wz && z == nz - 1) ? T(0) : u0[(int64_t)wrap_inc(z, nz) * sxy + (int64_t)y * sx + x];
        lap += ((zm_ - T(2) * c) + zp_) * inv_h2;
    }
    const T a = (c2 ? c2[idx] : c2_const) * lap;
    // U^{-1} = U^0 - dt V^0 + (dt^2/2) A(U^0)
    const T v = v0 ? v0[idx] : T(0);
    um1[idx] = (c - dt * v) + half_dt2 * a;
}

// Point sources: U[cell_s] += amp * w[s][n]   (amp = dt^2 / h^d).  The host
// sorts the sources by cell: cells[q] is the q-th cell in sorted order and
// order[q] the caller's index of that source.  The first thread of each run
// of equal cells adds the whole run (in the caller's order), so coincident
// sources need no atomics and the result is deterministic.
template <typename T>
__global__ void __launch_bounds__(256) k_inject(T *__restrict__ u, const int64_t *__restrict__ cells,
                                                const int64_t *__restrict__ order,
                                                const T *__restrict__ wav, int64_t ns, int64_t nt,
                                                int64_t n, T amp)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    const int64_t cell = cells[q];
    if (q > 0 && cells[q - 1] == cell) return;
    T add = T(0);
    for (int64_t r = q; r < ns && cells[r] == cell; ++r) add += wav[order[r] * nt + n];
    u[cell] += amp * add;
}

// Receivers: traces[r][n] = U[cell_r].
template <typename T>
__global__ void __launch_bounds__(256) k_record(const T *__restrict__ u, const int64_t *__restrict__ cells,
                                                T *__restrict__ traces, int64_t nr, int64_t nt, int64_t n)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    traces[r * nt + n] = u[cells[r]];
}

// Plane recorder: out[q] = U on the plane i_axis = index, q in x-fastest order
// of the two remaining axes (extents e0 fastest, e1).
template <typename T>
__global__ void __launch_bounds__(256) k_record_plane(const T *__restrict__ u, T *__restrict__ out,
                                                      int64_t e0, int64_t e1, int64_t s0, int64_t s1,
                                                      int64_t offset)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= e0 * e1) return;
    const int64_t a = q % e0, b = q / e0;
    out[q] = u[offset + a * s0 + b * s1];
}

// Non-finite scan: flags[block] = 1 if the block's cells hold a NaN or Inf.
template <typename T>
__global__ void __launch_bounds__(256) k_nonfinite(const T *__restrict__ u, int64_t n, int32_t *__restrict__ flags)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T v = u[i];
        bad |= !(v - v == T(0));   // NaN or +-Inf
    }
    if (bad) any = 1;              // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = any;
}

// ---------------------------------------------------------------------------
// Discrete adjoint of one step (transpose of the step map), reverse time.
// With a^k the adjoint of U^k and p_a, q_a those of Phi_a, Psi_a at level n+1:
//   a^n     = 2 a^{n+1} - a^{n+2} + dt^2 L(c^2 a^{n+1}) + dt sum_a G_a(p_a + q_a)
//   p_a^n   = p_a - dt/2 sigma(i)  (p_a(i) + p_a(i+e)) - dt^2/h sigma(i)   a^{n+1}(i+e)
//   q_a^n   = q_a - dt/2 sigma(i-1)(q_a(i) + q_a(i-e)) + dt^2/h sigma(i-1) a^{n+1}(i-e)
//   grad_c2 += dt^2 a^{n+1} (L U^n)           (summed over batch members in FP64)
// G_a U = (U(i+e) - U(i-e))/(2h), L the periodic Laplacian.  p_a is kept at
// band slots [0, M-1] and q_a at [1, M]; the other slot of each stays 0, so
// (p+q) can be read at any slot j <= M.  a^n overwrites a^{n+2} in place.
// ---------------------------------------------------------------------------
template <typename T>
struct AdjArgs {
    Axis<T> ax[3];    // sig; phi/psi = p, q at n+1; phi_o/psi_o = p, q at n
    const T *lam;     // a^{n+1}
    T *lam_o;         // a^{n+2}
    T *lam_w;         // where a^n goes: lam_o (in place) or another buffer
    const T *un;      // U^n
    const T *c2;      // per-cell c^2 or nullptr
    double *grad;     // dJ/dc^2, accumulated (+=), one value per cell
    T c2_const;       // c^2 when c2 == nullptr
    T inv_h2;         // 1 / h^2
    T inv_2h;         // 1 / (2h)
    T dt;             // dt
    T dt2;            // dt * dt
    T half_dt;        // dt / 2
    T k_damp;         // dt^2 / h
    int32_t nx, ny, nz, batch;
    int64_t bstride;
    int64_t bstride_aux[3];
    const TileRef *tiles;  // optional 64 x 4 tile list (2D) instead of the whole grid
    int32_t ntiles;
    int32_t skip[4];       // with a tile list: cells in [skip0, skip1) x [skip2, skip3) are left alone
    int32_t gskip[4];      // with a tile list: cells in [gskip0, gskip1) x [gskip2, gskip3) add no gradient
                           // (their gradient term is another kernel's)
};

// (p + q) of axis A at band slot j (0 outside the band).
template <typename T>
__device__ __forceinline__ T pq_at(const Axis<T> &A, int j, int64_t cbase, int64_t cstr, int64_t boff)
{
    if (A.M == 0 || j > A.M) return T(0);
    const int64_t c = boff + cbase + (int64_t)j * cstr;
    return A.phi[c] + A.psi[c];
}

// Geometry of one cell for the transposed step: flat index, neighbours,
// c^2 there (shared by all batch members) and per-axis band slots.
template <typename T>
struct AdjGeo {
    int64_t idx, nb[6];
    T cc, cn[6];
    int jc[3], jm[3], jp[3];
    int64_t cbase[3], cstr[3];
};

template <typename T, int D>
__device__ __forceinline__ AdjGeo<T> adj_geo(const AdjArgs<T> &p, int x, int y, int z)
{
    AdjGeo<T> g;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    g.idx = (int64_t)z * sz + (int64_t)y * sy + x;
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    const int zm = D == 3 ? wrap_dec(z, nz) : 0, zp = D == 3 ? wrap_inc(z, nz) : 0;
    g.nb[0] = g.idx - x + xm;
    g.nb[1] = g.idx - x + xp;
    g.nb[2] = g.idx + (int64_t)(ym - y) * sy;
    g.nb[3] = g.idx + (int64_t)(yp - y) * sy;
    g.nb[4] = g.idx + (int64_t)(zm - z) * sz;
    g.nb[5] = g.idx + (int64_t)(zp - z) * sz;
    g.cc = p.c2 ? p.c2[g.idx] : p.c2_const;
#pragma unroll
    for (int k = 0; k < 6; ++k) g.cn[k] = (k < 2 * D) ? (p.c2 ? p.c2[g.nb[k]] : p.c2_const) : T(0);
    const int coord[3] = {x, y, z};
    const int cm_[3] = {xm, ym, zm};
    const int cp_[3] = {xp, yp, zp};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Axis<T> &A = p.ax[a];
        g.jc[a] = g.jm[a] = g.jp[a] = 1 << 30;
        g.cbase[a] = 0;
        g.cstr[a] = 1;
        if (a < D && A.M > 0) {
            g.jc[a] = band_coord(A, coord[a]);
            g.jm[a] = band_coord(A, cm_[a]);
            g.jp[a] = band_coord(A, cp_[a]);
            if (a == 0) { g.cbase[a] = ((int64_t)z * ny + y) * (A.M + 1); g.cstr[a] = 1; }
            if (a == 1) { g.cbase[a] = (int64_t)z * (A.M + 1) * nx + x; g.cstr[a] = nx; }
            if (a == 2) { g.cbase[a] = (int64_t)y * nx + x; g.cstr[a] = (int64_t)nx * ny; }
        }
    }
    return g;
}

// What the transposed step of one shot reads at a cell: a^{n+1} and U^n at
// the cell and its neighbours, a^{n+2} at the cell, and per axis the
// adjoint auxiliaries at the neighbours' band slots (p and q apart) and at
// the cell's own slot and the slot beside it.
template <typename T>
struct AdjIn {
    T lc, uc, lo, ln[6], uu[6];
    T upp[3], upq[3], dnp[3], dnq[3];
    T pc[3], pr[3], qc[3], ql[3];
};

template <typename T, int D>
__device__ __forceinline__ void adj_load(const AdjArgs<T> &p, const AdjGeo<T> &g, int bi, AdjIn<T> &in)
{
    const int64_t bo = (int64_t)bi * p.bstride;
    const T *lam = p.lam + bo;
    const T *un = p.un + bo;
    in.lc = lam[g.idx];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        in.ln[k] = (k < 2 * D) ? lam[g.nb[k]] : T(0);
        in.uu[k] = (k < 2 * D) ? un[g.nb[k]] : T(0);
    }
    in.uc = un[g.idx];
    in.lo = p.lam_o[bo + g.idx];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const Axis<T> &A = p.ax[a];
        in.upp[a] = in.upq[a] = in.dnp[a] = in.dnq[a] = T(0);
        in.pc[a] = in.pr[a] = in.qc[a] = in.ql[a] = T(0);
        if (A.M == 0) continue;
        const int64_t ba = (int64_t)bi * p.bstride_aux[a] + g.cbase[a];
        if (g.jp[a] <= A.M) {
            const int64_t c = ba + (int64_t)g.jp[a] * g.cstr[a];
            in.upp[a] = A.phi[c];
            in.upq[a] = A.psi[c];
        }
        if (g.jm[a] <= A.M) {
            const int64_t c = ba + (int64_t)g.jm[a] * g.cstr[a];
            in.dnp[a] = A.phi[c];
            in.dnq[a] = A.psi[c];
        }
        if (g.jc[a] <= A.M) {
            const int j = g.jc[a];
            const int64_t c = ba + (int64_t)j * g.cstr[a];
            if (j < A.M) {
                in.pc[a] = A.phi[c];
                in.pr[a] = A.phi[c + g.cstr[a]];
            }
            if (j > 0) {
                in.qc[a] = A.psi[c];
                in.ql[a] = A.psi[c - g.cstr[a]];
            }
        }
    }
}

// The transposed step of shot bi at a cell from its loads (reverse mode of
// Eqs. (DiscretePML a-c)): writes a^n and the adjoint auxiliaries and
// returns the shot's c^2-gradient term.
template <typename T, int D>
__device__ __forceinline__ double adj_finish(const AdjArgs<T> &p, const AdjGeo<T> &g, int bi, const AdjIn<T> &in)
{
    const int64_t bo = (int64_t)bi * p.bstride;
    const T clc = g.cc * in.lc;
    T lapc = T(0), lapu = T(0);
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
        if (k < 2 * D) {
            lapc += ((g.cn[k] * in.ln[k] - T(2) * clc) + g.cn[k + 1] * in.ln[k + 1]) * p.inv_h2;
            lapu += ((in.uu[k] - T(2) * in.uc) + in.uu[k + 1]) * p.inv_h2;
        }
    }
    T v = (T(2) * in.lc - in.lo) + p.dt2 * lapc;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const Axis<T> &A = p.ax[a];
        if (A.M == 0) continue;
        const int64_t ba = (int64_t)bi * p.bstride_aux[a] + g.cbase[a];
        // G_a(p + q) from the neighbours' band slots ((p + q) is 0 off the band)
        if (g.jm[a] <= A.M || g.jp[a] <= A.M) {
            const T up_ = g.jp[a] <= A.M ? in.upp[a] + in.upq[a] : T(0);
            const T dn_ = g.jm[a] <= A.M ? in.dnp[a] + in.dnq[a] : T(0);
            v += (p.dt * (up_ - dn_)) * p.inv_2h;
        }
        if (g.jc[a] <= A.M) {
            const int j = g.jc[a];
            const int64_t c = ba + (int64_t)j * g.cstr[a];
            const T s = A.sig[j];
            const T sl = j > 0 ? A.sig[j - 1] : T(0);
            if (j < A.M) {
                const T pc = in.pc[a], pr = in.pr[a];
                A.phi_o[c] = (pc - (p.half_dt * s) * (pc + pr)) - (p.k_damp * s) * in.ln[2 * a + 1];
            }
            if (j > 0) {
                const T qc = in.qc[a], ql = in.ql[a];
                A.psi_o[c] = (qc - (p.half_dt * sl) * (qc + ql)) + (p.k_damp * sl) * in.ln[2 * a];
            }
        }
    }
    p.lam_w[bo + g.idx] = v;
    return (double)(p.dt2 * in.lc) * (double)lapu;
}

// The transposed step at cell (x, y, z) for the shots bi0, bi0 + bstep, ...:
// their c^2-gradient terms summed in FP64 in shot order.
template <typename T, int D>
__device__ __forceinline__ double adj_cell(const AdjArgs<T> &p, int x, int y, int z, int bi0, int bstep)
{
    const AdjGeo<T> g = adj_geo<T, D>(p, x, y, z);
    double gsum = 0.0;
#pragma unroll 1
    for (int bi = bi0; bi < p.batch; bi += bstep) {
        AdjIn<T> in;
        adj_load<T, D>(p, g, bi, in);
        gsum += adj_finish<T, D>(p, g, bi, in);
    }
    return gsum;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_adjoint_cell(AdjArgs<T> p)
{
    // 1-D XCD-aware launch over 64 x 4 cell tiles (as the forward CELL kernel),
    // one thread per cell looping over all shots
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tiles_x = (p.nx + 63) / 64, tiles_y = (p.ny + 3) / 4;
    if (tile >= tiles_x * tiles_y * (D == 3 ? p.nz : 1)) return;
    const int z = D == 3 ? tile / (tiles_x * tiles_y) : 0;
    const int rem = tile - z * tiles_x * tiles_y;
    const int x = (rem % tiles_x) * 64 + (int)(threadIdx.x % 64);
    const int y = (rem / tiles_x) * 4 + (int)(threadIdx.x / 64);
    if (x >= p.nx || y >= p.ny) return;
    const double g = adj_cell<T, D>(p, x, y, z, 0, 1);
    p.grad[((int64_t)z * p.ny + y) * p.nx + x] += g;
}

// Raw buffer access: one descriptor per array (four scalar registers;
// descriptor word 3 of gfx9 for untyped data, the record limit the array's
// bytes) and a per-lane 32-bit byte offset plus a scalar one (a batch
// member's start), so an access needs no 64-bit address in vector
// registers.  The arrays such an access reaches stay below 4 GiB (the host
// checks).
using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ Rsrc array_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buf_ld(Rsrc r, uint32_t off, uint32_t soff)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}

template <typename T>
__device__ __forceinline__ void buf_st(Rsrc r, uint32_t off, uint32_t soff, T v)
{
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, off, soff, 0);
}

// Load / store through a base pointer plus a 32-bit byte offset: with a
// wave-uniform base the hardware adds a scalar base to a vector offset, so a
// run of loads from different rows shares one offset register.
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

template <typename T>
__device__ __forceinline__ void st_off(T *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

// A wave-uniform pointer taken through readfirstlane: a shot's array base
// then sits in a scalar pair and the lanes' offsets are shared by all
// shots, instead of the loop keeping a 64-bit per-lane address for every
// access of every shot it has in flight (two vector registers each).
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// The 2D frame of the adjoint (cells outside the marching core) over a list
// of 64 x 4 tiles: a block takes one row of 64 cells of a tile, and its NG
// waves split the shots (wave w takes shots w, w+NG, ...), so a frame cell's
// shot loop is NG times shorter; a wave issues the loads of SB of its shots
// before the arithmetic of any.  Every access is a shot's array base (one
// scalar pair per array) plus a 32-bit byte offset within the member that
// all shots share, so a member's field and each axis's compact auxiliaries
// must stay below 2^32 bytes (the host checks).  The expressions and their
// order are those of adj_finish.  The NG FP64 partial gradients of a cell
// (each summed in shot order) are added in LDS in a fixed order (no atomics).
// BUF: the same accesses through one buffer descriptor per array over all
// members (a member's start a scalar offset; the host takes this form when
// every array is below 4 GiB): no 64-bit address math per access and fewer
// vector registers (88 against 103 in FP32), the same results.
template <typename T, int NG, int SB, bool BUF>
__global__ void __launch_bounds__(64 * NG) k_adjoint_frame2d(AdjArgs<T> p)
{
    __shared__ double part[NG][64];
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int t = b >> 2, row = b & 3;
    // the wave index is uniform across the wave: with it in a scalar register
    // every shot's array bases are scalar too
    const int lane = (int)(threadIdx.x & 63), w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nx = p.nx, ny = p.ny;
    bool ok = t < p.ntiles;
    int x = 0, y = 0;
    if (ok) {
        const TileRef tl = p.tiles[t];
        x = tl.tx * 64 + lane;
        y = tl.ty * 4 + row;
        ok = x < nx && y < ny && !(x >= p.skip[0] && x < p.skip[1] && y >= p.skip[2] && y < p.skip[3]);
    }
    double gsum = 0.0;
    if (ok) {
        constexpr uint32_t E = sizeof(T);
        const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx), ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
        const uint32_t oc = (uint32_t)(y * nx + x) * E, oxm = (uint32_t)(y * nx + xm) * E;
        const uint32_t oxp = (uint32_t)(y * nx + xp) * E, oym = (uint32_t)(ym * nx + x) * E;
        const uint32_t oyp = (uint32_t)(yp * nx + x) * E;
        // c^2 at the cell and at x-1, x+1, y-1, y+1 (shared by the shots)
        const T cc = p.c2 ? ld_off(p.c2, oc) : p.c2_const;
        const T cn0 = p.c2 ? ld_off(p.c2, oxm) : p.c2_const;
        const T cn1 = p.c2 ? ld_off(p.c2, oxp) : p.c2_const;
        const T cn2 = p.c2 ? ld_off(p.c2, oym) : p.c2_const;
        const T cn3 = p.c2 ? ld_off(p.c2, oyp) : p.c2_const;
        const Axis<T> &AX = p.ax[0], &AY = p.ax[1];
        const int MX = AX.M, MY = AY.M;
        int jx = 1 << 30, jxm = 1 << 30, jxp = 1 << 30, jy = 1 << 30, jym = 1 << 30, jyp = 1 << 30;
        if (MX > 0) {
            jx = band_coord(AX, x);
            jxm = band_coord(AX, xm);
            jxp = band_coord(AX, xp);
        }
        if (MY > 0) {
            jy = band_coord(AY, y);
            jym = band_coord(AY, ym);
            jyp = band_coord(AY, yp);
        }
        // offsets in the compact layouts: x band [y][MX+1], y band [MY+1][x]
        const uint32_t xr = (uint32_t)(y * (MX + 1));
        const uint32_t oxj = (xr + (uint32_t)jx) * E, oxjm = (xr + (uint32_t)jxm) * E, oxjp = (xr + (uint32_t)jxp) * E;
        const uint32_t oyj = (uint32_t)(jy * nx + x) * E, oyjm = (uint32_t)(jym * nx + x) * E;
        const uint32_t oyjp = (uint32_t)(jyp * nx + x) * E, orow = (uint32_t)nx * E;
        // BUF: one descriptor per array over all members, a member's start a
        // scalar offset (every array below 4 GiB)
        const uint32_t mb = (uint32_t)p.bstride * E, mbx = (uint32_t)p.bstride_aux[0] * E;
        const uint32_t mby = (uint32_t)p.bstride_aux[1] * E, nb = (uint32_t)p.batch;
        const Rsrc rl = array_rsrc(p.lam, nb * mb), ru = array_rsrc(p.un, nb * mb), ro = array_rsrc(p.lam_o, nb * mb);
        const Rsrc rw = array_rsrc(p.lam_w, nb * mb);
        const Rsrc rxp = array_rsrc(AX.phi, nb * mbx), rxq = array_rsrc(AX.psi, nb * mbx);
        const Rsrc rxpo = array_rsrc(AX.phi_o, nb * mbx), rxqo = array_rsrc(AX.psi_o, nb * mbx);
        const Rsrc ryp = array_rsrc(AY.phi, nb * mby), ryq = array_rsrc(AY.psi, nb * mby);
        const Rsrc rypo = array_rsrc(AY.phi_o, nb * mby), ryqo = array_rsrc(AY.psi_o, nb * mby);
#pragma unroll 1
        for (int b0 = w; b0 < p.batch; b0 += NG * SB) {
            T lc[SB], uc[SB], lo[SB], ln[SB][4], uu[SB][4];
            T xup[SB], xuq[SB], xdp[SB], xdq[SB], xpc[SB], xpr[SB], xqc[SB], xql[SB];
            T yup[SB], yuq[SB], ydp[SB], ydq[SB], ypc[SB], ypr[SB], yqc[SB], yql[SB];
#pragma unroll
            for (int k = 0; k < SB; ++k) {
                const int bi = b0 + k * NG;
                if (bi >= p.batch) break;
                xup[k] = xuq[k] = xdp[k] = xdq[k] = xpc[k] = xpr[k] = xqc[k] = xql[k] = T(0);
                yup[k] = yuq[k] = ydp[k] = ydq[k] = ypc[k] = ypr[k] = yqc[k] = yql[k] = T(0);
                if constexpr (BUF) {
                    const uint32_t so = (uint32_t)bi * mb;
                    lc[k] = buf_ld<T>(rl, oc, so);
                    ln[k][0] = buf_ld<T>(rl, oxm, so);
                    ln[k][1] = buf_ld<T>(rl, oxp, so);
                    ln[k][2] = buf_ld<T>(rl, oym, so);
                    ln[k][3] = buf_ld<T>(rl, oyp, so);
                    uc[k] = buf_ld<T>(ru, oc, so);
                    uu[k][0] = buf_ld<T>(ru, oxm, so);
                    uu[k][1] = buf_ld<T>(ru, oxp, so);
                    uu[k][2] = buf_ld<T>(ru, oym, so);
                    uu[k][3] = buf_ld<T>(ru, oyp, so);
                    lo[k] = buf_ld<T>(ro, oc, so);
                    if (MX > 0) {
                        const uint32_t sa = (uint32_t)bi * mbx;
                        if (jxp <= MX) { xup[k] = buf_ld<T>(rxp, oxjp, sa); xuq[k] = buf_ld<T>(rxq, oxjp, sa); }
                        if (jxm <= MX) { xdp[k] = buf_ld<T>(rxp, oxjm, sa); xdq[k] = buf_ld<T>(rxq, oxjm, sa); }
                        if (jx < MX) { xpc[k] = buf_ld<T>(rxp, oxj, sa); xpr[k] = buf_ld<T>(rxp, oxj + E, sa); }
                        if (jx > 0 && jx <= MX) { xqc[k] = buf_ld<T>(rxq, oxj, sa); xql[k] = buf_ld<T>(rxq, oxj - E, sa); }
                    }
                    if (MY > 0) {
                        const uint32_t sa = (uint32_t)bi * mby;
                        if (jyp <= MY) { yup[k] = buf_ld<T>(ryp, oyjp, sa); yuq[k] = buf_ld<T>(ryq, oyjp, sa); }
                        if (jym <= MY) { ydp[k] = buf_ld<T>(ryp, oyjm, sa); ydq[k] = buf_ld<T>(ryq, oyjm, sa); }
                        if (jy < MY) { ypc[k] = buf_ld<T>(ryp, oyj, sa); ypr[k] = buf_ld<T>(ryp, oyj + orow, sa); }
                        if (jy > 0 && jy <= MY) { yqc[k] = buf_ld<T>(ryq, oyj, sa); yql[k] = buf_ld<T>(ryq, oyj - orow, sa); }
                    }
                } else {
                    const int64_t bo = (int64_t)bi * p.bstride;
                    const T *lam = uniform_ptr(p.lam + bo), *un = uniform_ptr(p.un + bo);
                    lc[k] = ld_off(lam, oc);
                    ln[k][0] = ld_off(lam, oxm);
                    ln[k][1] = ld_off(lam, oxp);
                    ln[k][2] = ld_off(lam, oym);
                    ln[k][3] = ld_off(lam, oyp);
                    uc[k] = ld_off(un, oc);
                    uu[k][0] = ld_off(un, oxm);
                    uu[k][1] = ld_off(un, oxp);
                    uu[k][2] = ld_off(un, oym);
                    uu[k][3] = ld_off(un, oyp);
                    lo[k] = ld_off(uniform_ptr((const T *)p.lam_o + bo), oc);
                    if (MX > 0) {
                        const int64_t ba = (int64_t)bi * p.bstride_aux[0];
                        const T *ph = uniform_ptr(AX.phi + ba), *ps = uniform_ptr(AX.psi + ba);
                        if (jxp <= MX) { xup[k] = ld_off(ph, oxjp); xuq[k] = ld_off(ps, oxjp); }
                        if (jxm <= MX) { xdp[k] = ld_off(ph, oxjm); xdq[k] = ld_off(ps, oxjm); }
                        if (jx < MX) { xpc[k] = ld_off(ph, oxj); xpr[k] = ld_off(ph, oxj + E); }
                        if (jx > 0 && jx <= MX) { xqc[k] = ld_off(ps, oxj); xql[k] = ld_off(ps, oxj - E); }
                    }
                    if (MY > 0) {
                        const int64_t ba = (int64_t)bi * p.bstride_aux[1];
                        const T *ph = uniform_ptr(AY.phi + ba), *ps = uniform_ptr(AY.psi + ba);
                        if (jyp <= MY) { yup[k] = ld_off(ph, oyjp); yuq[k] = ld_off(ps, oyjp); }
                        if (jym <= MY) { ydp[k] = ld_off(ph, oyjm); ydq[k] = ld_off(ps, oyjm); }
                        if (jy < MY) { ypc[k] = ld_off(ph, oyj); ypr[k] = ld_off(ph, oyj + orow); }
                        if (jy > 0 && jy <= MY) { yqc[k] = ld_off(ps, oyj); yql[k] = ld_off(ps, oyj - orow); }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < SB; ++k) {
                const int bi = b0 + k * NG;
                if (bi >= p.batch) break;
                const int64_t bo = (int64_t)bi * p.bstride;
                const T clc = cc * lc[k];
                T lapc = T(0), lapu = T(0);
                lapc += ((cn0 * ln[k][0] - T(2) * clc) + cn1 * ln[k][1]) * p.inv_h2;
                lapu += ((uu[k][0] - T(2) * uc[k]) + uu[k][1]) * p.inv_h2;
                lapc += ((cn2 * ln[k][2] - T(2) * clc) + cn3 * ln[k][3]) * p.inv_h2;
                lapu += ((uu[k][2] - T(2) * uc[k]) + uu[k][3]) * p.inv_h2;
                T v = (T(2) * lc[k] - lo[k]) + p.dt2 * lapc;
                if (MX > 0) {
                    const int64_t ba = (int64_t)bi * p.bstride_aux[0];
                    if (jxm <= MX || jxp <= MX) {
                        const T up_ = jxp <= MX ? xup[k] + xuq[k] : T(0);
                        const T dn_ = jxm <= MX ? xdp[k] + xdq[k] : T(0);
                        v += (p.dt * (up_ - dn_)) * p.inv_2h;
                    }
                    if (jx <= MX) {
                        const T s = AX.sig[jx];
                        const T sl = jx > 0 ? AX.sig[jx - 1] : T(0);
                        if (jx < MX) {
                            const T vp = (xpc[k] - (p.half_dt * s) * (xpc[k] + xpr[k])) - (p.k_damp * s) * ln[k][1];
                            if constexpr (BUF) buf_st<T>(rxpo, oxj, (uint32_t)bi * mbx, vp);
                            else st_off(uniform_ptr(AX.phi_o + ba), oxj, vp);
                        }
                        if (jx > 0) {
                            const T vq = (xqc[k] - (p.half_dt * sl) * (xqc[k] + xql[k])) + (p.k_damp * sl) * ln[k][0];
                            if constexpr (BUF) buf_st<T>(rxqo, oxj, (uint32_t)bi * mbx, vq);
                            else st_off(uniform_ptr(AX.psi_o + ba), oxj, vq);
                        }
                    }
                }
                if (MY > 0) {
                    const int64_t ba = (int64_t)bi * p.bstride_aux[1];
                    if (jym <= MY || jyp <= MY) {
                        const T up_ = jyp <= MY ? yup[k] + yuq[k] : T(0);
                        const T dn_ = jym <= MY ? ydp[k] + ydq[k] : T(0);
                        v += (p.dt * (up_ - dn_)) * p.inv_2h;
                    }
                    if (jy <= MY) {
                        const T s = AY.sig[jy];
                        const T sl = jy > 0 ? AY.sig[jy - 1] : T(0);
                        if (jy < MY) {
                            const T vp = (ypc[k] - (p.half_dt * s) * (ypc[k] + ypr[k])) - (p.k_damp * s) * ln[k][3];
                            if constexpr (BUF) buf_st<T>(rypo, oyj, (uint32_t)bi * mby, vp);
                            else st_off(uniform_ptr(AY.phi_o + ba), oyj, vp);
                        }
                        if (jy > 0) {
                            const T vq = (yqc[k] - (p.half_dt * sl) * (yqc[k] + yql[k])) + (p.k_damp * sl) * ln[k][2];
                            if constexpr (BUF) buf_st<T>(ryqo, oyj, (uint32_t)bi * mby, vq);
                            else st_off(uniform_ptr(AY.psi_o + ba), oyj, vq);
                        }
                    }
                }
                if constexpr (BUF) buf_st<T>(rw, oc, (uint32_t)bi * mb, v);
                else st_off(uniform_ptr(p.lam_w + bo), oc, v);
                gsum += (double)(p.dt2 * lc[k]) * (double)lapu;
            }
        }
    }
    part[w][lane] = gsum;
    __syncthreads();
    if (ok && w == 0 && !(x >= p.gskip[0] && x < p.gskip[1] && y >= p.gskip[2] && y < p.gskip[3])) {
        double g = part[0][lane];
#pragma unroll
        for (int k = 1; k < NG; ++k) g += part[k][lane];
        p.grad[(int64_t)y * p.nx + x] += g;
    }
}

// Marching form of the same transposed step on the core of a 2D periodic
// grid -- the cells [cx0, cx1) x [cy0, cy1) whose update and neighbours
// carry no layer term (k_adjoint_cell takes the rest): each wave owns 64
// columns x R rows.  For every shot it issues the loads of its whole tile
// at once (rows -1..R of a^{n+1} and U^n, rows 0..R-1 of a^{n+2}, and the
// column beyond each strip edge), takes x neighbours from the adjacent lanes
// and y neighbours from the adjacent rows, and keeps the FP64 c^2 gradient
// of its R cells in registers across the shots (same order as the cell
// kernel: shots ascending, one add into grad at the end).  The expressions
// are those of k_adjoint_cell, evaluated in the same order.
template <typename T, int R>
__global__ void __launch_bounds__(256) k_adjoint_march2d(AdjArgs<T> p, int cx0, int cx1, int cy0, int cy1,
                                                         int tiles_x, int n_waves)
{
    // the wave index is uniform across the wave: keep it (and every row
    // index derived from it) in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny;
    const int tx = w % tiles_x, ty = w / tiles_x;
    const int x0 = cx0 + tx * 64, x = x0 + lane, y0 = cy0 + ty * R;
    const bool xout = x < cx1;                               // this lane's cell is the kernel's
    const int xc = x % nx;                                   // lanes past the edge read a wrapped column
    const int xe = lane == 0 ? (x0 - 1 + nx) % nx : (x0 + 64) % nx;   // lanes 0 / 63: outer column
    const bool edge = lane == 0 || lane == 63;
    constexpr uint32_t E = sizeof(T);
    const uint32_t oc = (uint32_t)xc * E, oe = (uint32_t)xe * E;
    // row y0-1+r (wrapped) as an element offset of the row start
    auto rowoff = [&](int r) -> int64_t {
        int y = y0 - 1 + r;
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        return (int64_t)y * nx;
    };
    // c^2 of the column (rows -1..R) and of the outer columns (edge lanes)
    T cl[R + 2], ce[R];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) cl[r] = p.c2 ? ld_off(p.c2 + rowoff(r), oc) : p.c2_const;
#pragma unroll
    for (int r = 0; r < R; ++r) ce[r] = (p.c2 && edge) ? ld_off(p.c2 + rowoff(r + 1), oe) : p.c2_const;
    double g[R];
#pragma unroll
    for (int r = 0; r < R; ++r) g[r] = 0.0;
#pragma unroll 1
    for (int bi = 0; bi < p.batch; ++bi) {
        const int64_t bo = (int64_t)bi * p.bstride;
        const T *lam = p.lam + bo, *un = p.un + bo;
        const T *lamo = p.lam_o + bo;
        T *lamw = p.lam_w + bo;
        T L[R + 2], U[R + 2], LO[R], LE[R], UE[R];
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            L[r] = ld_off(lam + rowoff(r), oc);
            U[r] = ld_off(un + rowoff(r), oc);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            LO[r] = ld_off(lamo + rowoff(r + 1), oc);
            LE[r] = UE[r] = T(0);
            if (edge) {
                LE[r] = ld_off(lam + rowoff(r + 1), oe);
                UE[r] = ld_off(un + rowoff(r + 1), oe);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (y0 + r >= cy1) break;                        // uniform
            const T lc = L[r + 1], uc = U[r + 1];
            const T clc = cl[r + 1] * lc;
            // neighbours across lanes (every lane shuffles; the edge lanes then
            // take the outer column): c^2 a and U of columns x-1 and x+1
            T cxm = __shfl_up(clc, 1), cxp = __shfl_down(clc, 1);
            T uxm = __shfl_up(uc, 1), uxp = __shfl_down(uc, 1);
            if (lane == 0) { cxm = ce[r] * LE[r]; uxm = UE[r]; }
            if (lane == 63) { cxp = ce[r] * LE[r]; uxp = UE[r]; }
            T lapc = T(0), lapu = T(0);
            lapc += ((cxm - T(2) * clc) + cxp) * p.inv_h2;
            lapu += ((uxm - T(2) * uc) + uxp) * p.inv_h2;
            lapc += ((cl[r] * L[r] - T(2) * clc) + cl[r + 2] * L[r + 2]) * p.inv_h2;
            lapu += ((U[r] - T(2) * uc) + U[r + 2]) * p.inv_h2;
            const T v = (T(2) * lc - LO[r]) + p.dt2 * lapc;
            if (xout) st_off(lamw + rowoff(r + 1), oc, v);
            g[r] += (double)(p.dt2 * lc) * (double)lapu;
        }
    }
    if (!xout) return;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (y0 + r < cy1) p.grad[(int64_t)(y0 + r) * nx + x] += g[r];
}

// Two transposed steps (n, then n-1) per pass on a 2D core r = [cx0, cx1) x
// [cy0, cy1) whose cells, and the cells one step around them, carry no layer
// term.  Each wave owns 62 columns (lanes 1..62; lanes 0 and 63 carry the
// halo, each loading the column beyond it) x R rows and loops over the
// shots.  Per shot it loads a^{n+1} on rows -2..R+1, a^{n+2}, U^n and U^{n-1}
// on rows -1..R, forms a^n on rows -1..R of every lane (adding the residual
// of step n-1 at receiver cells, as the step's injection would), then
// a^{n-1} on its own cells from those, in registers.  a^n is stored on r
// shrunk by one (the frame's first step writes the ring), a^{n-1} on r.  The
// FP64 c^2 gradient terms of both steps are kept per cell across the shots
// and added to grad one step after the other, as two single steps add them.
// The expressions are those of k_adjoint_march2d, in the same order.
template <typename T>
struct Adj2 {
    const T *un2;                  // U^{n-1}
    T *out1, *out2;                // a^n, a^{n-1}
    const int32_t *rmap;           // [member * ny + y]: pool slot of row y's column map, or -1 (nullptr: none)
    const int32_t *rpool;          // pool[slot + x]: receiver index of column x, or -1
    const T *resid;                // [nr][nt]
    int64_t nt, t;                 // residual columns; the column injected into a^n (n - 1; -1: none)
    int32_t s1[4];                 // the rectangle a^n is stored on (the frame writes the rest)
};

template <typename T, int R>
__global__ void __launch_bounds__(256) k_adjoint2_march2d(AdjArgs<T> p, Adj2<T> q, int cx0, int cx1, int cy0, int cy1,
                                                          int tiles_x, int n_waves)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (w >= n_waves) return;                                // whole waves; no barriers below
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny;
    const int tx = w % tiles_x, ty = w / tiles_x;
    const int x0 = cx0 + tx * 62 - 1, x = x0 + lane, y0 = cy0 + ty * R;
    const bool own = lane >= 1 && lane <= 62 && x < cx1;      // a^{n-1} and the gradient of this lane's cells
    const bool in1 = own && x >= q.s1[0] && x < q.s1[1];       // a^n stored (off r's ring on a layer axis)
    const int xc = (x + nx) % nx;                            // lanes past either edge read a wrapped column
    const int xe = lane == 0 ? (x0 - 1 + nx) % nx : (x0 + 64) % nx;   // lanes 0 / 63: outer column
    const bool edge = lane == 0 || lane == 63;
    constexpr uint32_t E = sizeof(T);
    const uint32_t oc = (uint32_t)xc * E, oe = (uint32_t)xe * E;
    // row y0 - 2 + r (wrapped) as an element offset of the row start
    auto rowoff = [&](int r) -> int64_t {
        int y = y0 - 2 + r;
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        return (int64_t)y * nx;
    };
    // c^2 of the column (rows -2..R+1) and of the outer columns (rows -1..R)
    T cl[R + 4], ce[R + 2];
#pragma unroll
    for (int r = 0; r < R + 4; ++r) cl[r] = p.c2 ? ld_off(p.c2 + rowoff(r), oc) : p.c2_const;
#pragma unroll
    for (int r = 0; r < R + 2; ++r) ce[r] = (p.c2 && edge) ? ld_off(p.c2 + rowoff(r + 1), oe) : p.c2_const;
    double g1[R], g2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) g1[r] = g2[r] = 0.0;
    // receiver columns of rows -1..R of this member (set per shot)
#pragma unroll 1
    for (int bi = 0; bi < p.batch; ++bi) {
        const int64_t bo = (int64_t)bi * p.bstride;
        const T *lam = p.lam + bo, *lamo = p.lam_o + bo, *un = p.un + bo, *un2 = q.un2 + bo;
        T L[R + 4], LE[R + 2], LO[R + 2], U1[R + 2], U2[R + 2];
#pragma unroll
        for (int r = 0; r < R + 4; ++r) L[r] = ld_off(lam + rowoff(r), oc);
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            LO[r] = ld_off(lamo + rowoff(r + 1), oc);
            U1[r] = ld_off(un + rowoff(r + 1), oc);
            U2[r] = ld_off(un2 + rowoff(r + 1), oc);
            LE[r] = edge ? ld_off(lam + rowoff(r + 1), oe) : T(0);
        }
        // a^n on rows -1..R (index r + 1), every lane
        T V[R + 2];
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const T lc = L[r + 1];
            const T clc = cl[r + 1] * lc;
            T cxm = __shfl_up(clc, 1), cxp = __shfl_down(clc, 1);
            if (lane == 0) cxm = ce[r] * LE[r];
            if (lane == 63) cxp = ce[r] * LE[r];
            T lapc = T(0);
            lapc += ((cxm - T(2) * clc) + cxp) * p.inv_h2;
            lapc += ((cl[r] * L[r] - T(2) * clc) + cl[r + 2] * L[r + 2]) * p.inv_h2;
            T v = (T(2) * lc - LO[r]) + p.dt2 * lapc;
            if (q.rmap && q.t >= 0) {
                int y = y0 - 1 + r;
                y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
                const int slot = q.rmap[(int64_t)bi * ny + y];    // uniform
                if (slot >= 0) {
                    const int ri = q.rpool[slot + xc];
                    if (ri >= 0) {
                        const T add = T(0) + q.resid[(int64_t)ri * q.nt + q.t];
                        v += T(1) * add;
                    }
                }
            }
            V[r] = v;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (y0 + r >= cy1) break;                        // uniform
            // step n on row r: gradient from a^{n+1} and U^n; a^n stored off the ring
            {
                const T lc = L[r + 2], uc = U1[r + 1];
                T uxm = __shfl_up(uc, 1), uxp = __shfl_down(uc, 1);
                T lapu = T(0);
                lapu += ((uxm - T(2) * uc) + uxp) * p.inv_h2;
                lapu += ((U1[r] - T(2) * uc) + U1[r + 2]) * p.inv_h2;
                g1[r] += (double)(p.dt2 * lc) * (double)lapu;
                const int y = y0 + r;
                if (in1 && y >= q.s1[2] && y < q.s1[3]) st_off(q.out1 + bo + rowoff(r + 2), oc, V[r + 1]);
            }
            // step n-1 on row r from a^n (registers) and a^{n+1}
            const T lc = V[r + 1], uc = U2[r + 1];
            const T clc = cl[r + 2] * lc;
            T cxm = __shfl_up(clc, 1), cxp = __shfl_down(clc, 1);
            T uxm = __shfl_up(uc, 1), uxp = __shfl_down(uc, 1);
            T lapc = T(0), lapu = T(0);
            lapc += ((cxm - T(2) * clc) + cxp) * p.inv_h2;
            lapu += ((uxm - T(2) * uc) + uxp) * p.inv_h2;
            lapc += ((cl[r + 1] * V[r] - T(2) * clc) + cl[r + 3] * V[r + 2]) * p.inv_h2;
            lapu += ((U2[r] - T(2) * uc) + U2[r + 2]) * p.inv_h2;
            const T v = (T(2) * lc - L[r + 2]) + p.dt2 * lapc;
            if (own) st_off(q.out2 + bo + rowoff(r + 2), oc, v);
            g2[r] += (double)(p.dt2 * lc) * (double)lapu;
        }
    }
    if (!own) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (y0 + r >= cy1) break;
        double *gc = p.grad + (int64_t)(y0 + r) * nx + x;
        *gc += g1[r];
        *gc += g2[r];
    }
}

// Adjoint of the start U^{-1} = U^0 + dt^2/2 c^2 L U^0 with a^{-1} = -a^1:
// grad_c2 += dt^2/2 (-a^1) (L U^0), summed over batch members.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_adjoint_start(const T *__restrict__ a1, const T *__restrict__ u0,
                                                       double *__restrict__ grad, T half_dt2, T inv_h2,
                                                       int nx, int ny, int nz, int batch, int64_t bstride)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = D == 3 ? (int)blockIdx.z : 0;
    if (x >= nx || y >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t idx = (int64_t)z * sz + (int64_t)y * sy + x;
    double g = 0.0;
    for (int bi = 0; bi < batch; ++bi) {
        const T *u = u0 + (int64_t)bi * bstride;
        const T c = u[idx];
        T lap = T(0);
        lap += ((u[idx - x + wrap_dec(x, nx)] - T(2) * c) + u[idx - x + wrap_inc(x, nx)]) * inv_h2;
        lap += ((u[idx + (int64_t)(wrap_dec(y, ny) - y) * sy] - T(2) * c) + u[idx + (int64_t)(wrap_inc(y, ny) - y) * sy]) * inv_h2;
        if (D == 3)
            lap += ((u[idx + (int64_t)(wrap_dec(z, nz) - z) * sz] - T(2) * c) + u[idx + (int64_t)(wrap_inc(z, nz) - z) * sz]) * inv_h2;
        g += (double)(half_dt2 * -a1[(int64_t)bi * bstride + idx]) * (double)lap;
    }
    grad[idx] += g;
}

// out[order[q] * nt + n] = amp * u[cells[q]]  (gather, e.g. the wavelet gradient).
template <typename T>
__global__ void __launch_bounds__(256) k_gather_scaled(const T *__restrict__ u, const int64_t *__restrict__ cells,
                                                       const int64_t *__restrict__ order, T *__restrict__ out,
                                                       int64_t count, int64_t nt, int64_t n, T amp)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    out[order[q] * nt + n] = amp * u[cells[q]];
}

// ---------------------------------------------------------------------------
// The paper's own integrator: classic RK4 on (U, V = U_t, Phi_a, Psi_a) with
// the right-hand sides of Eq. (DiscretePML a, b, c).  One launch per stage:
//   k      = f(Y_in)                       (Y_in = Y0 at stage 0)
//   S      = w_0 k (stage 0), S + w_s k (stages 1, 2)
//   Y_out  = Y0 + (c_{s+1} dt) k           (stages 0..2)
//   Y_new  = Y0 + dt (S + w_3 k)           (stage 3, written over S)
// with c = (0, 1/2, 1/2, 1), w = (1/6, 2/6, 2/6, 1/6).
// ---------------------------------------------------------------------------
template <typename T>
struct RKFields {
    T *u, *v;
    T *phi[3], *psi[3];
};

template <typename T>
struct RKArgs {
    Axis<T> ax[3];          // sig and geometry only
    RKFields<T> yin, y0, s, yout;
    const T *c2;
    T c2_const, inv_h2, inv_h, inv_2h;
    T w;                    // w_s
    T w3;                   // w_3 (stage 3)
    T cdt;                  // c_{s+1} dt (stages 0..2)
    T dt;
    int32_t stage;
    int32_t nx, ny, nz;
};

template <typename T, int D>
__global__ void __launch_bounds__(256) k_rk4_stage(RKArgs<T> p)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = D == 3 ? (int)blockIdx.z : 0;
    if (x >= p.nx || y >= p.ny) return;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t idx = (int64_t)z * sz + (int64_t)y * sy + x;
    const int coord[3] = {x, y, z};
    const int64_t stride[3] = {1, sy, sz};
    const int ext[3] = {nx, ny, nz};
    const T *U = p.yin.u;
    const T uc = U[idx];
    T lap = T(0), damp = T(0);
    T dphi[3] = {T(0), T(0), T(0)}, dpsi[3] = {T(0), T(0), T(0)};
    int jj[3] = {1 << 30, 1 << 30, 1 << 30};
    int64_t cidx[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int i = coord[a];
        const int64_t cm = idx + (int64_t)(wrap_dec(i, ext[a]) - i) * stride[a];
        const int64_t cp = idx + (int64_t)(wrap_inc(i, ext[a]) - i) * stride[a];
        const T um = U[cm], up = U[cp];
        lap += ((um - T(2) * uc) + up) * p.inv_h2;
        const Axis<T> &A = p.ax[a];
        if (A.M > 0) {
            const int j = band_coord(A, i);
            if (j <= A.M) {
                int64_t base, cstr;
                if (a == 0) { base = ((int64_t)z * ny + y) * (A.M + 1); cstr = 1; }
                else if (a == 1) { base = (int64_t)z * (A.M + 1) * nx + x; cstr = nx; }
                else { base = (int64_t)y * nx + x; cstr = (int64_t)nx * ny; }
                const int64_t c = base + (int64_t)j * cstr;
                const T *phi = p.yin.phi[a], *psi = p.yin.psi[a];
                const T sg = A.sig[j];
                const T sl = j > 0 ? A.sig[j - 1] : T(0);
                const T phi_l = j > 0 ? phi[c - cstr] : T(0);
                const T psi_r = j < A.M ? psi[c + cstr] : T(0);
                damp += (sg * psi_r - sl * phi_l) * p.inv_h;
                const T grad = (up - um) * p.inv_2h;
                dphi[a] = T(-0.5) * (sl * phi_l + sg * phi[c]) - grad;
                dpsi[a] = T(-0.5) * (sl * psi[c] + sg * psi_r) - grad;
                jj[a] = j;
                cidx[a] = c;
            }
        }
    }
    const T ku = p.yin.v[idx];
    const T kv = (p.c2 ? p.c2[idx] : p.c2_const) * lap + damp;
    // combine one field value: k is its derivative, c its index
    auto combine = [&](const T *y0, T *sacc, T *yout, int64_t c, T k) {
        if (p.stage == 0) sacc[c] = p.w * k;
        else if (p.stage < 3) sacc[c] = sacc[c] + p.w * k;
        else sacc[c] = y0[c] + p.dt * (sacc[c] + p.w3 * k);
        if (p.stage < 3) yout[c] = y0[c] + p.cdt * k;
    };
    combine(p.y0.u, p.s.u, p.yout.u, idx, ku);
    combine(p.y0.v, p.s.v, p.yout.v, idx, kv);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int j = jj[a];
        if (j > p.ax[a].M) continue;
        if (j < p.ax[a].M) combine(p.y0.phi[a], p.s.phi[a], p.yout.phi[a], cidx[a], dphi[a]);
        if (j > 0) combine(p.y0.psi[a], p.s.psi[a], p.yout.psi[a], cidx[a], dpsi[a]);
    }
}

}  // namespace dpmlk
