// dpml_kernels3d.hpp -- gfx950 z-marching kernels of one 3D step over a box,
// with the layer terms of Eq. (DiscretePML a-c) taken from register
// neighbours.
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

}  // namespace dpmlk
