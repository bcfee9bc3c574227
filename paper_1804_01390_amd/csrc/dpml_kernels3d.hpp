// dpml_kernels3d.hpp -- gfx950 z-marching kernels of one 3D step over a box,
// with the layer terms of Eq. (DiscretePML a-c) taken from register
// neighbours, and (at the end of the file) the frame of a 3D two-step pass
// taken as two levels per march.
//
// A wave owns a strip of 64 consecutive columns (lanes 1..62 produce, lanes
// 0 and 63 only feed their neighbours) and RY consecutive rows, and marches
// through a chunk of planes in +z.  At plane k it holds U^n of planes k-1, k
// for its rows in registers and has the loads of the next PF planes in
// flight (U^n of plane k+1, U^{n-1} of plane k, the two halo rows of plane
// k, and the layer inputs of plane k).  Neighbours come from registers:
//   x  cross-lane DPP row shifts (the strip's halo lanes);
//   y  the adjacent register rows (the halo rows y0-1, y0+RY from memory);
//   z  the previous / next plane of the march.
// The layer terms reuse the same structure, so each auxiliary value is read
// once per step:
//   Phi_x(i-e), Psi_x(i+e)  from the neighbouring lanes (compact layout
//                            [z][y][Mx+1]: the band lanes read consecutive slots);
//   Phi_y(i-e), Psi_y(i+e)  from the adjacent register rows ([z][My+1][x]), the
//                            wave's first/last row reading one slot beyond;
//   Phi_z(i-e)               kept from the previous plane, Psi_z(i+e) loaded with
//                            the next plane ([Mz+1][y][x]).
// Every cell evaluates the expressions of cell_update (dpml_kernels.hpp) in
// the same order, so results are bit-identical to the other step kernels.
//
// AX is the set of axes whose layer terms the box's cells may meet (bit a for
// axis a).  The library splits a step into boxes -- the layer-free core
// (AX = 0), the x-band strip (1), the z-band slab (5) and the y-band slab
// (7) -- so each launch carries only the registers its cells need.
// Periodic axes only (walls take the other step kernels).
#pragma once

#include "dpml_kernels.hpp"

namespace dpmlk {

// A box of output cells: columns [xs, xe), rows [ys, ye), planes [zs, ze),
// each start inside the array and each extent at most the axis length;
// indices past the array end continue at its start (the periodic wrap, so
// the two halves of a layer band form one box).  Waves: `strips` strips of
// 62 output columns x `groups` groups of RY rows x `chunks` chunks of
// `chunk` planes, the row group varying fastest.
struct MBox {
    int32_t xs, xe, ys, ye, zs, ze;
    int32_t strips, groups, chunk, chunks;
};

template <typename T, int RY, int AX>
struct MFetch {
    static constexpr int NXL = (AX & 1) ? RY : 1;
    static constexpr int NYL = (AX & 2) ? RY : 1;
    static constexpr int NZL = (AX & 4) ? RY : 1;
    T up[RY];          // U^n, plane k+1
    T old[RY];         // U^{n-1}, plane k
    T hlo, hhi;        // U^n, plane k, rows y0-1 and y0+RY
    T fx[NXL], qx[NXL];// Phi_x, Psi_x of plane k (band lanes)
    T fy[NYL], qy[NYL];// Phi_y, Psi_y of plane k (band rows)
    T fyl, qyh;        // Phi_y of row y0-1, Psi_y of row y0+RY (band slots beyond the wave)
    T fz[NZL], qz1[NZL];// Phi_z of plane k, Psi_z of plane k+1
};

// Streaming loads and stores: U^{n-1} is read once and U^{n+1} written once
// per step, so with NT they bypass the caches' normal retention (non-temporal
// hints), leaving the cache to the U^n rows and planes the neighbours share.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// One wave's march over its part of box bx: wave index `wave` within the box
// (row group fastest, then strip, then chunk).
template <typename T, int RY, int PF, int AX, bool NT>
__device__ __forceinline__ void march_box(StepArgs<T> p, const MBox &bx, int wave)
{
    using F = MFetch<T, RY, AX>;
    const int per_chunk = bx.strips * bx.groups;
    const int ck = wave / per_chunk;
    if (ck >= bx.chunks) return;                        // whole wave; no barriers below
    const int rem = wave - ck * per_chunk;
    const int st = rem / bx.groups;
    const int gr = rem - st * bx.groups;
    select_member(p, (int)blockIdx.y);
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t sxy = (int64_t)nx * ny;
    // columns: lane l holds column xs + 62 st + l - 1 (unwrapped, >= -1)
    const int xu = bx.xs + 62 * st + lane - 1;
    const int xc = xu < 0 ? xu + nx : (xu >= nx ? xu - nx : xu);
    const bool xout = lane >= 1 && lane <= 62 && xu < bx.xe;
    const bool xneed = xu <= bx.xe;                     // feeds an output column
    const uint32_t xo = (uint32_t)xc;
    // rows y0 .. y0+RY-1 (all loaded; rows at or past ye are not stored)
    const int y0 = bx.ys + gr * RY;
    int ry[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) ry[q] = (y0 + q) % ny;
    const int rlo = (y0 + ny - 1) % ny, rhi = (y0 + RY) % ny;
    const int nrow = min(RY, bx.ye - y0);               // rows stored
    auto wrapz = [&](int z) { return z >= nz ? z - nz : z; };
    const int z0 = bx.zs + ck * bx.chunk;
    const int z1 = min(z0 + bx.chunk, bx.ze);
    const T *u = p.u;
    const T *uo_in = p.uo;
    T *out = p.uout ? p.uout : p.uo;
    auto row_ptr = [&](const T *b, int z, int r) -> const T * { return b + ((int64_t)z * sxy + (int64_t)r * nx); };

    // ---- layer geometry ----------------------------------------------------
    const Axis<T> &Ax = p.ax[0], &Ay = p.ax[1], &Az = p.ax[2];
    // x: the lane's band slot and damping (constant along the march)
    int jx = 1 << 30;
    T sx = T(0), sxl = T(0);
    bool lx = false;
    if constexpr ((AX & 1) != 0) {
        if (Ax.M > 0) {
            jx = band_coord(Ax, xc);
            lx = jx <= Ax.M && xneed;
            if (lx) {
                sx = Ax.sig[jx];
                sxl = jx > 0 ? Ax.sig[jx - 1] : T(0);
            }
        }
    }
    // y: band slot of each row (wave-uniform)
    int jy[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) jy[q] = 1 << 30;
    if constexpr ((AX & 2) != 0) {
        if (Ay.M > 0) {
#pragma unroll
            for (int q = 0; q < RY; ++q) jy[q] = band_coord(Ay, ry[q]);
        }
    }
    const int64_t xstr_y = (int64_t)(Ay.M + 1) * nx;   // plane stride of the compact y arrays
    auto zslot = [&](int zc) -> int {
        if constexpr ((AX & 4) != 0) return Az.M > 0 ? band_coord(Az, zc) : (1 << 30);
        return 1 << 30;
    };

    // ---- loads of plane k ----------------------------------------------------
    auto fetch = [&](int k, F &f) {
        const int kc = wrapz(k), kn = wrapz(k + 1);
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            f.up[q] = xneed ? row_ptr(u, kn, ry[q])[xo] : T(0);
            f.old[q] = xneed ? ld_stream<NT>(row_ptr(uo_in, kc, ry[q]) + xo) : T(0);
        }
        f.hlo = xneed ? row_ptr(u, kc, rlo)[xo] : T(0);
        f.hhi = xneed ? row_ptr(u, kc, rhi)[xo] : T(0);
        if constexpr ((AX & 1) != 0) {
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                f.fx[q] = T(0);
                f.qx[q] = T(0);
                if (lx) {
                    const int64_t c = ((int64_t)kc * ny + ry[q]) * (Ax.M + 1) + jx;
                    f.fx[q] = Ax.phi[c];
                    f.qx[q] = Ax.psi[c];
                }
            }
        }
        if constexpr ((AX & 2) != 0) {
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                f.fy[q] = T(0);
                f.qy[q] = T(0);
                if (jy[q] <= Ay.M && xneed) {
                    const int64_t c = (int64_t)kc * xstr_y + (int64_t)jy[q] * nx + xc;
                    f.fy[q] = Ay.phi[c];
                    f.qy[q] = Ay.psi[c];
                }
            }
            // Phi_y one slot below the first row, Psi_y one slot beyond the last
            f.fyl = T(0);
            f.qyh = T(0);
            if (jy[0] >= 1 && jy[0] <= Ay.M && xneed) f.fyl = Ay.phi[(int64_t)kc * xstr_y + (int64_t)(jy[0] - 1) * nx + xc];
            if (jy[RY - 1] < Ay.M && xneed)
                f.qyh = Ay.psi[(int64_t)kc * xstr_y + (int64_t)(jy[RY - 1] + 1) * nx + xc];
        }
        if constexpr ((AX & 4) != 0) {
            const int jk = zslot(kc), jn = zslot(kn);
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                f.fz[q] = T(0);
                f.qz1[q] = T(0);
                if (jk <= Az.M && xneed) f.fz[q] = Az.phi[((int64_t)jk * ny + ry[q]) * nx + xc];
                if (jn <= Az.M && xneed) f.qz1[q] = Az.psi[((int64_t)jn * ny + ry[q]) * nx + xc];
            }
        }
    };

    // ---- march ---------------------------------------------------------------
    T um[RY], uc[RY];
    T pzl[(AX & 4) ? RY : 1], qzc[(AX & 4) ? RY : 1];   // Phi_z of plane k-1, Psi_z of plane k
    {
        const int zc = wrapz(z0), zm = zc == 0 ? nz - 1 : zc - 1;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            um[q] = xneed ? row_ptr(u, zm, ry[q])[xo] : T(0);
            uc[q] = xneed ? row_ptr(u, zc, ry[q])[xo] : T(0);
        }
        if constexpr ((AX & 4) != 0) {
            const int jm = zslot(zm), jc = zslot(zc);
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                pzl[q] = (jm <= Az.M && xneed) ? Az.phi[((int64_t)jm * ny + ry[q]) * nx + xc] : T(0);
                qzc[q] = (jc <= Az.M && xneed) ? Az.psi[((int64_t)jc * ny + ry[q]) * nx + xc] : T(0);
            }
        }
    }
    F fq[PF + 1];
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (z0 + i < z1) fetch(z0 + i, fq[i]);
    const T inv_h2 = p.inv_h2, inv_h = p.inv_h, inv_2h = p.inv_2h, dt = p.dt, dt2 = p.dt2;
    for (int k = z0; k < z1; ++k) {
        if (k + PF < z1) fetch(k + PF, fq[PF]);
        F &f = fq[0];
        const int kc = wrapz(k);
        const int64_t plane = (int64_t)kc * sxy;
        const int jz = zslot(kc);
        const bool lz = (AX & 4) != 0 && jz <= Az.M;
        T szv = T(0), szl = T(0);
        if constexpr ((AX & 4) != 0) {
            if (lz) {
                szv = Az.sig[jz];
                szl = jz > 0 ? Az.sig[jz - 1] : T(0);
            }
        }
        // x-neighbour shifts of the x-layer inputs (all lanes take part)
        T fxl[(AX & 1) ? RY : 1], qxr[(AX & 1) ? RY : 1];
        if constexpr ((AX & 1) != 0) {
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                fxl[q] = from_left(f.fx[q]);
                qxr[q] = from_right(f.qx[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            const T c0 = uc[q];
            const T uxm = from_left(c0), uxp = from_right(c0);
            const T uym = q == 0 ? f.hlo : uc[q - 1];
            const T uyp = q == RY - 1 ? f.hhi : uc[q + 1];
            const T uzm = um[q], uzp = f.up[q];
            const int64_t idx = plane + (int64_t)ry[q] * nx + xc;
            const bool store = xout && q < nrow;
            const T c2 = p.c2 ? (store ? p.c2[idx] : T(1)) : p.c2_const;
            T lap = ((uxm - T(2) * c0) + uxp) * inv_h2;
            lap += ((uym - T(2) * c0) + uyp) * inv_h2;
            lap += ((uzm - T(2) * c0) + uzp) * inv_h2;
            T damp = T(0);
            if constexpr ((AX & 1) != 0) {
                if (lx) {
                    const T phl = jx > 0 ? fxl[q] : T(0);
                    const T psr = jx < Ax.M ? qxr[q] : T(0);
                    const T grad = (uxp - uxm) * inv_2h;
                    const int64_t c = ((int64_t)kc * ny + ry[q]) * (Ax.M + 1) + jx;
                    if (store && jx < Ax.M)
                        Ax.phi_o[c] = f.fx[q] + dt * (T(-0.5) * (sxl * phl + sx * f.fx[q]) - grad);
                    if (store && jx > 0)
                        Ax.psi_o[c] = f.qx[q] + dt * (T(-0.5) * (sxl * f.qx[q] + sx * psr) - grad);
                    damp += (sx * psr - sxl * phl) * inv_h;
                }
            }
            if constexpr ((AX & 2) != 0) {
                const int j = jy[q];
                if (j <= Ay.M) {
                    const T s = Ay.sig[j], sl = j > 0 ? Ay.sig[j - 1] : T(0);
                    const T phl = j > 0 ? (q == 0 ? f.fyl : f.fy[q - 1]) : T(0);
                    const T psr = j < Ay.M ? (q == RY - 1 ? f.qyh : f.qy[q + 1]) : T(0);
                    const T grad = (uyp - uym) * inv_2h;
                    const int64_t c = (int64_t)kc * xstr_y + (int64_t)j * nx + xc;
                    if (store && j < Ay.M)
                        Ay.phi_o[c] = f.fy[q] + dt * (T(-0.5) * (sl * phl + s * f.fy[q]) - grad);
                    if (store && j > 0)
                        Ay.psi_o[c] = f.qy[q] + dt * (T(-0.5) * (sl * f.qy[q] + s * psr) - grad);
                    damp += (s * psr - sl * phl) * inv_h;
                }
            }
            if constexpr ((AX & 4) != 0) {
                if (lz) {
                    const T phl = jz > 0 ? pzl[q] : T(0);
                    const T psr = jz < Az.M ? f.qz1[q] : T(0);
                    const T grad = (uzp - uzm) * inv_2h;
                    const int64_t c = ((int64_t)jz * ny + ry[q]) * nx + xc;
                    if (store && jz < Az.M)
                        Az.phi_o[c] = f.fz[q] + dt * (T(-0.5) * (szl * phl + szv * f.fz[q]) - grad);
                    if (store && jz > 0)
                        Az.psi_o[c] = qzc[q] + dt * (T(-0.5) * (szl * qzc[q] + szv * psr) - grad);
                    damp += (szv * psr - szl * phl) * inv_h;
                }
            }
            const T rhs = c2 * lap + damp;
            const T r = (T(2) * c0 - f.old[q]) + dt2 * rhs;
            if (store) {
                st_stream<NT>(out + idx, r);
                if (p.hist) p.hist[idx] = r;
            }
        }
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            um[q] = uc[q];
            uc[q] = f.up[q];
        }
        if constexpr ((AX & 4) != 0) {
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                pzl[q] = f.fz[q];
                qzc[q] = f.qz1[q];
            }
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) fq[i] = fq[i + 1];
    }
}

// One box per launch.
template <typename T, int RY, int PF, int AX, bool NT>
__global__ void __launch_bounds__(256) k_march3d(StepArgs<T> p, MBox bx)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    march_box<T, RY, PF, AX, NT>(p, bx, xcd_tile(blockIdx.x, gridDim.x) * 4 + wv);
}

// A whole step in one launch: the y-band box (rows of one wave each, all
// layer code), the z-band and x-band boxes (RYL rows per wave; x and z, or x
// layer code) and the layer-free core (RYC rows per wave, no layer code);
// each wave finds its box from the wave offsets.  Tiles go in launch order
// (the XCDs interleaved), so at any time the whole GPU marches through one
// stretch of the wave order: the same chunk of planes.  CF = 0 puts the
// layer boxes' waves first, CF = 1 the core's.
struct MPlan {
    MBox b[4];         // y band, z band, x band, core (empty boxes have no waves)
    int32_t w[4];      // cumulative wave counts in launch order
};

template <typename T, int RYC, int RYL, bool CF>
__global__ void __launch_bounds__(256) k_march3d_plan(StepArgs<T> p, MPlan pl)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int wave = (int)blockIdx.x * 4 + wv;
    if constexpr (CF) {
        const int nc = pl.w[3] - pl.w[2];
        if (wave < nc) {
            march_box<T, RYC, 1, 0, false>(p, pl.b[3], wave);
            return;
        }
        wave -= nc;
    }
    if (wave < pl.w[0]) march_box<T, 1, 1, 7, false>(p, pl.b[0], wave);
    else if (wave < pl.w[1]) march_box<T, RYL, 1, 5, false>(p, pl.b[1], wave - pl.w[0]);
    else if (wave < pl.w[2]) march_box<T, RYL, 1, 1, false>(p, pl.b[2], wave - pl.w[1]);
    else if (!CF && wave < pl.w[3]) march_box<T, RYC, 1, 0, false>(p, pl.b[3], wave - pl.w[2]);
}

// ---------------------------------------------------------------------------
// The frame of a 3D two-step pass as two levels in one launch: every cell
// outside the core box, layer terms included.  A wave holds 64 consecutive
// columns (two halo lanes per side, 60 produce) x RY rows and marches through
// a chunk of planes.  At march plane k it forms level one on plane k -- U^{n+1}
// on the rows -1 .. RY and the auxiliaries of level n+1 that the second level
// reads -- from level-n data, then level two (U^{n+2} and the auxiliaries of
// level n+2) on plane k-1 from the level-one values held in registers.  Per
// cell it reads U^n, U^{n-1} and the layer arrays of level n once and writes
// U^{n+1}, U^{n+2} and the layer arrays of level n+2 (into the aux buffer it
// did not read): the auxiliaries of level n+1 never reach memory.  Neighbours
// of the level-one auxiliaries: Phi_x(i-e), Psi_x(i+e) from the adjacent
// lanes; Phi_y one row below and Psi_y one row beyond each row (level one
// forms Phi_y on the rows -1 .. RY-1 and Psi_y on 0 .. RY); Phi_z of the
// previous and Psi_z of the next march plane.  Both levels evaluate
// cell_update's expressions in its order, so results are bit-identical to
// single steps.  Constant c^2, periodic axes, one batch member.
// ---------------------------------------------------------------------------
template <typename T, int RY, int AX>
struct F2Fetch {
    static constexpr int NR = RY + 2;
    static constexpr int NXA = (AX & 1) ? NR : 1;
    static constexpr int NYA = (AX & 2) ? NR + 1 : 1;
    static constexpr int NZA = (AX & 4) ? NR : 1;
    T up[NR];             // U^n, plane k+1, rows -1 .. RY
    T old[NR];            // U^{n-1}, plane k, rows -1 .. RY
    T hlo, hhi;           // U^n, plane k, rows -2 and RY+1
    T fx[NXA], qx[NXA];   // Phi_x^n, Psi_x^n of plane k, rows -1 .. RY (band lanes)
    T fy[NYA];            // Phi_y^n of plane k, rows -2 .. RY
    T qy[NYA];            // Psi_y^n of plane k, rows -1 .. RY+1
    T fz[NZA];            // Phi_z^n of plane k, rows -1 .. RY
    T qz1[NZA];           // Psi_z^n of plane k+1, rows -1 .. RY
};

// One wave's two-level march over its part of box bx (output cells; row
// group fastest, then strip of 60 columns, then chunk of planes).  out1,
// out2 receive U^{n+1}, U^{n+2} on the box's cells.  PA: the layer arrays of
// the next plane are loaded a plane ahead with U (more registers), else at
// the start of their own plane.
template <typename T, int RY, int AX, bool PA>
__device__ __forceinline__ void frame2_box(const StepArgs<T> &p, T *__restrict__ out1, T *__restrict__ out2,
                                           const MBox &bx, int wave)
{
    using F = F2Fetch<T, RY, AX>;
    constexpr int NR = RY + 2;
    constexpr bool LX = (AX & 1) != 0, LY = (AX & 2) != 0, LZ = (AX & 4) != 0;
    const int per_chunk = bx.strips * bx.groups;
    const int ck = wave / per_chunk;
    if (ck >= bx.chunks) return;                         // whole wave; no barriers below
    const int rem = wave - ck * per_chunk;
    const int st = rem / bx.groups;
    const int gr = rem - st * bx.groups;
    const int lane = (int)(threadIdx.x & 63);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t sxy = (int64_t)nx * ny;
    const int xu = bx.xs - 2 + 60 * st + lane;          // unwrapped column, >= -2
    const int xc = ((xu % nx) + nx) % nx;
    const bool need = xu < bx.xe + 2;                   // lanes past the reach read nothing
    const bool xout = lane >= 2 && lane < 62 && xu < bx.xe;
    const uint32_t xo = (uint32_t)xc;
    const int y0 = bx.ys + gr * RY;                     // first output row (unwrapped)
    int ra[RY + 4];                                     // array rows of the relative rows -2 .. RY+1
#pragma unroll
    for (int t = 0; t < RY + 4; ++t) ra[t] = (((y0 - 2 + t) % ny) + ny) % ny;
    const int nrow = min(RY, bx.ye - y0);               // rows stored
    auto zw = [&](int k) -> int { return ((k % nz) + nz) % nz; };
    const int z0 = bx.zs + ck * bx.chunk;
    const int z1 = min(z0 + bx.chunk, bx.ze);
    const T *u = p.u;
    const T *uo = p.uo;
    auto ld = [&](const T *b, int zc, int row) -> T {
        const T *rp = b + ((int64_t)zc * sxy + (int64_t)row * nx);
        return need ? rp[xo] : T(0);
    };

    // ---- layer geometry ----------------------------------------------------
    const Axis<T> &Ax = p.ax[0], &Ay = p.ax[1], &Az = p.ax[2];
    int jx = 1 << 30;
    T sx = T(0), sxl = T(0);
    bool lx = false;
    if constexpr (LX) {
        if (Ax.M > 0) {
            jx = band_coord(Ax, xc);
            lx = jx <= Ax.M && need;
            if (lx) {
                sx = Ax.sig[jx];
                sxl = jx > 0 ? Ax.sig[jx - 1] : T(0);
            }
        }
    }
    // band slots of the rows -2 .. RY+1 (wave-uniform); along a band the slot
    // of the row below is one less, across the periodic wrap too
    int jy[RY + 4];
#pragma unroll
    for (int t = 0; t < RY + 4; ++t) jy[t] = 1 << 30;
    if constexpr (LY) {
        if (Ay.M > 0) {
#pragma unroll
            for (int t = 0; t < RY + 4; ++t) jy[t] = band_coord(Ay, ra[t]);
        }
    }
    const int64_t ystr = (int64_t)(Ay.M + 1) * nx;     // plane stride of the compact y arrays
    auto zslot = [&](int zc) -> int {
        if constexpr (LZ) return Az.M > 0 ? band_coord(Az, zc) : (1 << 30);
        return 1 << 30;
    };
    auto zidx = [&](int j, int row) -> int64_t { return ((int64_t)j * ny + row) * nx + xc; };

    // ---- loads of plane k: U, then the layer arrays -----------------------
    auto fetch_u = [&](int k, F &f) {
        const int kc = zw(k), kn = zw(k + 1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            f.up[i] = ld(u, kn, ra[i + 1]);
            f.old[i] = ld(uo, kc, ra[i + 1]);
        }
        f.hlo = ld(u, kc, ra[0]);
        f.hhi = ld(u, kc, ra[RY + 3]);
    };
    auto fetch_a = [&](int k, F &f) {
        const int kc = zw(k), kn = zw(k + 1);
        (void)kn;
        if constexpr (LX) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                f.fx[i] = T(0);
                f.qx[i] = T(0);
                if (lx) {
                    const int64_t c = ((int64_t)kc * ny + ra[i + 1]) * (Ax.M + 1) + jx;
                    f.fx[i] = Ax.phi[c];
                    f.qx[i] = Ax.psi[c];
                }
            }
        }
        if constexpr (LY) {
            // fy[t]: row t-2 (slot jy[t]); qy[t]: row t-1 (slot jy[t+1])
#pragma unroll
            for (int t = 0; t < NR + 1; ++t) {
                const int jf = jy[t], jq = jy[t + 1];
                f.fy[t] = (jf <= Ay.M && need) ? Ay.phi[(int64_t)kc * ystr + (int64_t)jf * nx + xc] : T(0);
                f.qy[t] = (jq <= Ay.M && need) ? Ay.psi[(int64_t)kc * ystr + (int64_t)jq * nx + xc] : T(0);
            }
        }
        if constexpr (LZ) {
            const int jk = zslot(kc), jn = zslot(kn);
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                f.fz[i] = (jk <= Az.M && need) ? Az.phi[zidx(jk, ra[i + 1])] : T(0);
                f.qz1[i] = (jn <= Az.M && need) ? Az.psi[zidx(jn, ra[i + 1])] : T(0);
            }
        }
    };

    // ---- march ---------------------------------------------------------------
    constexpr int RX = LX ? RY : 1, RYA = LY ? RY + 1 : 1, RZ = LZ ? RY : 1, NZR = LZ ? NR : 1;
    T n0[NR], n1[NR];            // U^n of planes k-1, k (rows -1 .. RY)
    T a0[RY], a1[NR];            // U^{n+1} of planes k-2 (rows 0 .. RY-1), k-1 (rows -1 .. RY)
    T pzl[NZR], qzc[NZR];        // Phi_z^n of plane k-1, Psi_z^n of plane k (rows -1 .. RY)
    T px1[RX], qx1[RX];          // Phi_x^{n+1}, Psi_x^{n+1} of plane k-1 (rows 0 .. RY-1)
    T py1[RYA];                  // Phi_y^{n+1} of plane k-1, rows -1 .. RY-1
    T qy1[RYA];                  // Psi_y^{n+1} of plane k-1, rows 0 .. RY
    T pz0[RZ], pz1[RZ], qz1v[RZ];// Phi_z^{n+1} of planes k-2, k-1; Psi_z^{n+1} of plane k-1
    {
        const int zm = zw(z0 - 2), zc = zw(z0 - 1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            n0[i] = ld(u, zm, ra[i + 1]);
            n1[i] = ld(u, zc, ra[i + 1]);
        }
        if constexpr (LZ) {
            const int jm = zslot(zm), jc = zslot(zc);
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                pzl[i] = (jm <= Az.M && need) ? Az.phi[zidx(jm, ra[i + 1])] : T(0);
                qzc[i] = (jc <= Az.M && need) ? Az.psi[zidx(jc, ra[i + 1])] : T(0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) a1[i] = T(0);
#pragma unroll
    for (int r = 0; r < RY; ++r) a0[r] = T(0);
#pragma unroll
    for (int r = 0; r < RX; ++r) px1[r] = qx1[r] = T(0);
#pragma unroll
    for (int r = 0; r < RYA; ++r) py1[r] = qy1[r] = T(0);
#pragma unroll
    for (int r = 0; r < RZ; ++r) pz0[r] = pz1[r] = qz1v[r] = T(0);
    const T inv_h2 = p.inv_h2, inv_h = p.inv_h, inv_2h = p.inv_2h, dt = p.dt, dt2 = p.dt2, c2c = p.c2_const;
    F cur;
    fetch_u(z0 - 1, cur);
    if constexpr (PA) fetch_a(z0 - 1, cur);
    for (int k = z0 - 1; k <= z1; ++k) {
        // the next plane's loads in flight during this plane's arithmetic (the
        // layer arrays too with PA; else they are loaded here for this plane)
        F nxt;
        if (k + 1 <= z1) {
            fetch_u(k + 1, nxt);
            if constexpr (PA) fetch_a(k + 1, nxt);
        }
        if constexpr (!PA) fetch_a(k, cur);
        const int kc = zw(k);
        // ---- level one: plane k, rows -1 .. RY ----
        const int jz = zslot(kc);
        const bool lz = LZ && jz <= Az.M;
        T szv = T(0), szl = T(0);
        if constexpr (LZ) {
            if (lz) {
                szv = Az.sig[jz];
                szl = jz > 0 ? Az.sig[jz - 1] : T(0);
            }
        }
        T fxl[LX ? NR : 1], qxr[LX ? NR : 1];
        if constexpr (LX) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                fxl[i] = from_left(cur.fx[i]);
                qxr[i] = from_right(cur.qx[i]);
            }
        }
        T a2[NR];
        T px2[RX], qx2[RX], py2[RYA], qy2[RYA], pz2[RZ], qz2[RZ];
#pragma unroll
        for (int i = 0; i < NR; ++i) {                  // relative row i-1
            const T uc = n1[i];
            const T uxm = from_left(uc), uxp = from_right(uc);
            const T uym = i == 0 ? cur.hlo : n1[i - 1];
            const T uyp = i == NR - 1 ? cur.hhi : n1[i + 1];
            const T uzm = n0[i], uzp = cur.up[i];
            T lap = ((uxm - T(2) * uc) + uxp) * inv_h2;
            lap += ((uym - T(2) * uc) + uyp) * inv_h2;
            lap += ((uzm - T(2) * uc) + uzp) * inv_h2;
            T damp = T(0);
            if constexpr (LX) {
                T f1 = T(0), q1 = T(0);
                if (lx) {
                    const T phl = jx > 0 ? fxl[i] : T(0);
                    const T psr = jx < Ax.M ? qxr[i] : T(0);
                    const T grad = (uxp - uxm) * inv_2h;
                    if (jx < Ax.M) f1 = cur.fx[i] + dt * (T(-0.5) * (sxl * phl + sx * cur.fx[i]) - grad);
                    if (jx > 0) q1 = cur.qx[i] + dt * (T(-0.5) * (sxl * cur.qx[i] + sx * psr) - grad);
                    damp += (sx * psr - sxl * phl) * inv_h;
                }
                if (i >= 1 && i <= RY) {
                    px2[i - 1] = f1;
                    qx2[i - 1] = q1;
                }
            }
            if constexpr (LY) {
                const int j = jy[i + 1];
                T f1 = T(0), q1 = T(0);
                if (j <= Ay.M) {
                    const T s = Ay.sig[j], sl = j > 0 ? Ay.sig[j - 1] : T(0);
                    const T phl = j > 0 ? cur.fy[i] : T(0);          // row i-2
                    const T psr = j < Ay.M ? cur.qy[i + 1] : T(0);   // row i
                    const T phc = cur.fy[i + 1], psc = cur.qy[i];
                    const T grad = (uyp - uym) * inv_2h;
                    if (j < Ay.M) f1 = phc + dt * (T(-0.5) * (sl * phl + s * phc) - grad);
                    if (j > 0) q1 = psc + dt * (T(-0.5) * (sl * psc + s * psr) - grad);
                    damp += (s * psr - sl * phl) * inv_h;
                }
                if (i <= RY) py2[i] = f1;                   // rows -1 .. RY-1
                if (i >= 1) qy2[i - 1] = q1;                // rows 0 .. RY
            }
            if constexpr (LZ) {
                T f1 = T(0), q1 = T(0);
                if (lz) {
                    const T phl = jz > 0 ? pzl[i] : T(0);
                    const T psr = jz < Az.M ? cur.qz1[i] : T(0);
                    const T grad = (uzp - uzm) * inv_2h;
                    if (jz < Az.M) f1 = cur.fz[i] + dt * (T(-0.5) * (szl * phl + szv * cur.fz[i]) - grad);
                    if (jz > 0) q1 = qzc[i] + dt * (T(-0.5) * (szl * qzc[i] + szv * psr) - grad);
                    damp += (szv * psr - szl * phl) * inv_h;
                }
                if (i >= 1 && i <= RY) {
                    pz2[i - 1] = f1;
                    qz2[i - 1] = q1;
                }
            }
            const T rhs = c2c * lap + damp;
            a2[i] = (T(2) * uc - cur.old[i]) + dt2 * rhs;
        }
        if (k >= z0 && k < z1) {
            const int64_t plane = (int64_t)kc * sxy;
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (xout && r < nrow) (out1 + (plane + (int64_t)ra[r + 2] * nx))[xo] = a2[r + 1];
        }
        // ---- level two: plane k-1, rows 0 .. RY-1 ----
        if (k >= z0 + 1) {
            const int zp = zw(k - 1);
            const int jp = zslot(zp);
            const bool lzp = LZ && jp <= Az.M;
            T spv = T(0), spl = T(0);
            if constexpr (LZ) {
                if (lzp) {
                    spv = Az.sig[jp];
                    spl = jp > 0 ? Az.sig[jp - 1] : T(0);
                }
            }
            T pxl[RX], qxr2[RX];
            if constexpr (LX) {
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    pxl[r] = from_left(px1[r]);
                    qxr2[r] = from_right(qx1[r]);
                }
            }
            const int64_t plane = (int64_t)zp * sxy;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const bool store = xout && r < nrow;
                const T uc = a1[r + 1];
                const T uxm = from_left(uc), uxp = from_right(uc);
                const T uym = a1[r], uyp = a1[r + 2];
                const T uzm = a0[r], uzp = a2[r + 1];
                T lap = ((uxm - T(2) * uc) + uxp) * inv_h2;
                lap += ((uym - T(2) * uc) + uyp) * inv_h2;
                lap += ((uzm - T(2) * uc) + uzp) * inv_h2;
                T damp = T(0);
                if constexpr (LX) {
                    if (lx) {
                        const T phl = jx > 0 ? pxl[r] : T(0);
                        const T psr = jx < Ax.M ? qxr2[r] : T(0);
                        const T grad = (uxp - uxm) * inv_2h;
                        const int64_t c = ((int64_t)zp * ny + ra[r + 2]) * (Ax.M + 1) + jx;
                        if (store && jx < Ax.M)
                            Ax.phi_o[c] = px1[r] + dt * (T(-0.5) * (sxl * phl + sx * px1[r]) - grad);
                        if (store && jx > 0)
                            Ax.psi_o[c] = qx1[r] + dt * (T(-0.5) * (sxl * qx1[r] + sx * psr) - grad);
                        damp += (sx * psr - sxl * phl) * inv_h;
                    }
                }
                if constexpr (LY) {
                    const int j = jy[r + 2];
                    if (j <= Ay.M) {
                        const T s = Ay.sig[j], sl = j > 0 ? Ay.sig[j - 1] : T(0);
                        const T phl = j > 0 ? py1[r] : T(0);          // row r-1
                        const T psr = j < Ay.M ? qy1[r + 1] : T(0);   // row r+1
                        const T phc = py1[r + 1], psc = qy1[r];
                        const T grad = (uyp - uym) * inv_2h;
                        const int64_t c = (int64_t)zp * ystr + (int64_t)j * nx + xc;
                        if (store && j < Ay.M) Ay.phi_o[c] = phc + dt * (T(-0.5) * (sl * phl + s * phc) - grad);
                        if (store && j > 0) Ay.psi_o[c] = psc + dt * (T(-0.5) * (sl * psc + s * psr) - grad);
                        damp += (s * psr - sl * phl) * inv_h;
                    }
                }
                if constexpr (LZ) {
                    if (lzp) {
                        const T phl = jp > 0 ? pz0[r] : T(0);
                        const T psr = jp < Az.M ? qz2[r] : T(0);
                        const T phc = pz1[r], psc = qz1v[r];
                        const T grad = (uzp - uzm) * inv_2h;
                        const int64_t c = zidx(jp, ra[r + 2]);
                        if (store && jp < Az.M) Az.phi_o[c] = phc + dt * (T(-0.5) * (spl * phl + spv * phc) - grad);
                        if (store && jp > 0) Az.psi_o[c] = psc + dt * (T(-0.5) * (spl * psc + spv * psr) - grad);
                        damp += (spv * psr - spl * phl) * inv_h;
                    }
                }
                const T rhs = c2c * lap + damp;
                const T v = (T(2) * uc - n0[r + 1]) + dt2 * rhs;
                if (store) (out2 + (plane + (int64_t)ra[r + 2] * nx))[xo] = v;
            }
        }
        // ---- shift the march ----
#pragma unroll
        for (int r = 0; r < RY; ++r) a0[r] = a1[r + 1];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            a1[i] = a2[i];
            n0[i] = n1[i];
            n1[i] = cur.up[i];
        }
        if constexpr (LX) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                px1[r] = px2[r];
                qx1[r] = qx2[r];
            }
        }
        if constexpr (LY) {
#pragma unroll
            for (int r = 0; r < RY + 1; ++r) {
                py1[r] = py2[r];
                qy1[r] = qy2[r];
            }
        }
        if constexpr (LZ) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                pz0[r] = pz1[r];
                pz1[r] = pz2[r];
                qz1v[r] = qz2[r];
            }
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                pzl[i] = cur.fz[i];
                qzc[i] = cur.qz1[i];
            }
        }
        cur = nxt;
    }
}

// One box of the two-level frame per launch (each box type with its own
// register allocation); blocks congruent mod 8 take consecutive waves, so
// neighbouring row groups share their halo rows in one XCD's L2.
template <typename T, int RY, int AX, bool PA>
__global__ void __launch_bounds__(256) k_frame2_box3d(StepArgs<T> p, T *__restrict__ out1, T *__restrict__ out2,
                                                      MBox bx)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    frame2_box<T, RY, AX, PA>(p, out1, out2, bx, xcd_tile(blockIdx.x, gridDim.x) * 4 + wv);
}

// The boxes outside the core along two or three axes (its edges and
// corners: few waves each) in one launch: a wave finds its box from the
// cumulative wave counts w (boxes with the layer code of x and y, x and z,
// y and z, all three).
struct F2Edges {
    MBox b[4];
    int32_t w[4];
};

template <typename T, bool PA>
__global__ void __launch_bounds__(256) k_frame2_edges3d(StepArgs<T> p, T *__restrict__ out1, T *__restrict__ out2,
                                                        F2Edges e)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wave = xcd_tile(blockIdx.x, gridDim.x) * 4 + wv;
    if (wave < e.w[0]) frame2_box<T, 2, 3, PA>(p, out1, out2, e.b[0], wave);
    else if (wave < e.w[1]) frame2_box<T, 2, 5, PA>(p, out1, out2, e.b[1], wave - e.w[0]);
    else if (wave < e.w[2]) frame2_box<T, 2, 6, PA>(p, out1, out2, e.b[2], wave - e.w[1]);
    else if (wave < e.w[3]) frame2_box<T, 2, 7, PA>(p, out1, out2, e.b[3], wave - e.w[2]);
}

}  // namespace dpmlk
