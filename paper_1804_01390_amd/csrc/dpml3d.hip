// dpml3d.hip -- 3D stepping paths of the discrete-PML wave stepper: the
// marching single steps split into boxes (layer-free core, x-band strip, y and
// z layer slabs) and the multi-step passes (a temporally blocked core beside
// the frame's single steps), their launch shapes and algorithmic byte counts.
// The per-cell arithmetic is Eq. (DiscretePML a-c) of Chern, "A Reflectionless
// Discrete Perfectly Matched Layer", as in dpml_kernels.hpp.
#include "dpml_host.hpp"
#include "dpml_kernels3d.hpp"

namespace dpmlh {

// Box of a 3D step where no y or z damping term acts: [lo+1, lo+n) on an
// axis with a layer (cell lo still meets sigma(lo-1)), the whole axis
// without one.  Returns {y0, y1, z0, z1}.
static void march_box3d(const Layout &L, int b[4])
{
    for (int a = 1; a < 3; ++a) {
        const int k = 2 * (a - 1);
        if (L.M[a] == 0) {
            b[k] = 0;
            b[k + 1] = (int)L.N[a];
        } else {
            b[k] = L.lo[a] + 1;
            b[k + 1] = (int)(L.lo[a] + L.n[a]);
        }
    }
}

// One thread-per-cell launch over a box with the layer code of the axes in
// `ax` (x and z, or all).
template <typename T>
int launch_box(dpml *H, dpmlk::StepArgs<T> p, const dpmlk::Box3 &bx, int ax, hipStream_t st, int kind,
               double bytes = -1)
{
    if (bx.xe <= bx.xs || bx.ye <= bx.ys || bx.ze <= bx.zs) return DPML_OK;
    p.tiles_x = (bx.xe - bx.xs + 63) / 64;
    p.tiles_y = (bx.ye - bx.ys + 3) / 4;
    p.n_tiles = p.tiles_x * p.tiles_y * (bx.ze - bx.zs);
    if (H->timing && bytes < 0) bytes = step_bytes(H, box_cells(bx), box_aux(H->L, bx));
    const int slot = H->timing ? timed_begin(H, kind, bytes, st) : -1;
    const dim3 grid((unsigned)round8(p.n_tiles), (unsigned)H->L.batch), block(256);
    if (ax == 5) hipLaunchKernelGGL((dpmlk::k_step_box3d<T, 5>), grid, block, 0, st, p, bx);
    else hipLaunchKernelGGL((dpmlk::k_step_box3d<T, 7>), grid, block, 0, st, p, bx);
    if (slot >= 0) timed_end(H, slot, st);
    return DPML_OK;
}

// One z-march launch over a box with the layer code of the axes in `ax`
// (none or x alone), `ry` register rows per wave and `zchunk` planes per
// tile.
template <typename T>
int launch_zmarch(dpml *H, dpmlk::StepArgs<T> p, const dpmlk::Box3 &bx, int ry, int ax, int zchunk,
                  hipStream_t st, int kind, double bytes = -1)
{
    if (bx.xe <= bx.xs || bx.ye <= bx.ys || bx.ze <= bx.zs) return DPML_OK;
    p.tile_rows = zchunk;
    p.tiles_x = (bx.xe - bx.xs + 63) / 64;
    p.tiles_y = (bx.ye - bx.ys + 4 * ry - 1) / (4 * ry);
    const int tz = (bx.ze - bx.zs + zchunk - 1) / zchunk;
    p.n_tiles = p.tiles_x * p.tiles_y * tz;
    if (H->timing && bytes < 0) bytes = step_bytes(H, box_cells(bx), box_aux(H->L, bx));
    const int slot = H->timing ? timed_begin(H, kind, bytes, st) : -1;
    const dim3 grid((unsigned)round8(p.n_tiles), (unsigned)H->L.batch), block(256);
#define DPML_ZMARCH(RY_, AX_) hipLaunchKernelGGL((dpmlk::k_step_zmarch3d<T, RY_, AX_>), grid, block, 0, st, p, bx)
    if (ry == 4) {
        if (ax == 0) DPML_ZMARCH(4, 0);
        else DPML_ZMARCH(4, 1);
    } else {
        if (ax == 0) DPML_ZMARCH(2, 0);
        else DPML_ZMARCH(2, 1);
    }
#undef DPML_ZMARCH
    if (slot >= 0) timed_end(H, slot, st);
    return DPML_OK;
}

// 3D marching step as boxes:
//   core    x strips [64 s0, 64 s1) that no x damping term reaches, rows and
//           planes [lo+1, lo+n) (the box of march_box3d): no layer code;
//   x band  the remaining columns [64 s1, 64 s0 + N) of the same rows and
//           planes (one box across the periodic wrap): x-layer code;
//   y band  every column and plane of the rows [lo+n, lo+n+M] (wrapped):
//           all layer code, one thread per cell;
//   z band  every column of the box's rows, planes [lo+n, lo+n+M]: x and z
//           layer code, one thread per cell.
// The boxes partition the grid.  The layer boxes run on the side stream
// while the core runs on the handle's stream; they write disjoint cells and
// the step ends with the handle's stream waiting for the side stream.
// Launch shape of the register-neighbour marching step (k_march3d_plan):
// bits 0-11 of tile_rows planes per chunk of the core's waves (0: 64), bits
// 12-15 rows per core wave (1, 2, 4 or 8; 0: 4), bits 16-17 rows per wave of
// the z-band and x-band boxes (0: 1, 1: 2, 2: 4), bit 18 the core's waves
// first in launch order (else the layer boxes'), bit 19 the core and the
// layer boxes as two launches on two streams (else one launch), bits 20-27
// planes per chunk of the layer waves (0: 16).
struct MShape {
    int chunk, ry, ryl, cf, split, lchunk;
};

static MShape mshape(int tile_rows)
{
    MShape s;
    s.chunk = (tile_rows & 0xFFF) ? (tile_rows & 0xFFF) : 64;
    const int ry = (tile_rows >> 12) & 0xF;
    s.ry = (ry == 1 || ry == 2 || ry == 8) ? ry : 4;
    const int yl = (tile_rows >> 16) & 3;
    s.ryl = yl == 1 ? 2 : (yl == 2 ? 4 : 1);
    s.cf = (tile_rows >> 18) & 1;
    s.split = (tile_rows >> 19) & 1;
    s.lchunk = ((tile_rows >> 20) & 0xFF) ? ((tile_rows >> 20) & 0xFF) : 16;
    return s;
}

static dpmlk::MBox make_mbox(const dpmlk::Box3 &bx, int ry, int chunk)
{
    dpmlk::MBox m{bx.xs, bx.xe, bx.ys, bx.ye, bx.zs, bx.ze, 0, 0, 1, 0};
    if (bx.xe <= bx.xs || bx.ye <= bx.ys || bx.ze <= bx.zs) return m;   // no waves
    m.strips = (bx.xe - bx.xs + 61) / 62;
    m.groups = (bx.ye - bx.ys + ry - 1) / ry;
    m.chunk = std::min(chunk, bx.ze - bx.zs);
    m.chunks = (bx.ze - bx.zs + m.chunk - 1) / m.chunk;
    return m;
}

static int64_t mbox_waves(const dpmlk::MBox &m) { return (int64_t)m.strips * m.groups * m.chunks; }

template <typename T, int RYC, int RYL>
static void plan_launch(bool cf, dim3 g, hipStream_t st, const dpmlk::StepArgs<T> &p, const dpmlk::MPlan &pl)
{
    if (cf) hipLaunchKernelGGL((dpmlk::k_march3d_plan<T, RYC, RYL, true>), g, dim3(256), 0, st, p, pl);
    else hipLaunchKernelGGL((dpmlk::k_march3d_plan<T, RYC, RYL, false>), g, dim3(256), 0, st, p, pl);
}

template <typename T, int RYC>
static void plan_launch_ryl(int ryl, bool cf, dim3 g, hipStream_t st, const dpmlk::StepArgs<T> &p,
                            const dpmlk::MPlan &pl)
{
    if (ryl == 4) plan_launch<T, RYC, 4>(cf, g, st, p, pl);
    else if (ryl == 2) plan_launch<T, RYC, 2>(cf, g, st, p, pl);
    else plan_launch<T, RYC, 1>(cf, g, st, p, pl);
}

// One k_march3d_plan launch over the boxes of `pl` (wave offsets filled in
// here); `bytes` is the algorithmic byte count it reports when timed.
template <typename T>
static int launch_plan(dpml *H, const dpmlk::StepArgs<T> &p, dpmlk::MPlan pl, const MShape &s, hipStream_t st,
                       int kind, double bytes)
{
    int64_t w = 0;
    for (int i = 0; i < 4; ++i) {
        w += mbox_waves(pl.b[i]);
        pl.w[i] = (int32_t)w;
    }
    if (w == 0) return DPML_OK;
    if (w > ((int64_t)1 << 30)) return H->fail(DPML_EINVAL, "3D grid too large for one marching launch");
    const dim3 g((unsigned)((w + 3) / 4), (unsigned)H->L.batch);
    const int slot = H->timing ? timed_begin(H, kind, bytes, st) : -1;
    if (s.ry == 8) plan_launch_ryl<T, 8>(s.ryl, s.cf, g, st, p, pl);
    else if (s.ry == 2) plan_launch_ryl<T, 2>(s.ryl, s.cf, g, st, p, pl);
    else if (s.ry == 1) plan_launch_ryl<T, 1>(s.ryl, s.cf, g, st, p, pl);
    else plan_launch_ryl<T, 4>(s.ryl, s.cf, g, st, p, pl);
    if (slot >= 0) timed_end(H, slot, st);
    return DPML_OK;
}

// 3D marching step of periodic grids by k_march3d_plan, as boxes that
// partition the grid (per axis a with a layer, "inner" = [lo+1, lo+n), the
// cells no a damping term reaches; an axis without a layer is inner over
// its whole extent):
//   y band  rows [lo+n, lo+n+M] (wrapped), every column and plane: all layer code;
//   z band  inner rows, planes [lo+n, lo+n+M], every column: x and z layer code;
//   x band  columns [lo+n, lo+n+M], inner rows and planes: x layer code;
//   core    inner columns, rows and planes: no layer code.
// By default all four boxes are one launch (the layer boxes' waves first);
// split shapes run the core on the handle's stream and the layer boxes as a
// second launch on the side stream beside it.
template <typename T>
static int launch_mstep3d(dpml *H, const dpmlk::StepArgs<T> &p, const MShape &s)
{
    const Layout &L = H->L;
    int in0[3], in1[3], bb[3];
    for (int a = 0; a < 3; ++a) {
        bb[a] = L.lo[a] + (int)L.n[a];
        if (L.M[a] == 0) {
            in0[a] = 0;
            in1[a] = (int)L.N[a];
        } else {
            in0[a] = L.lo[a] + 1;
            in1[a] = L.lo[a] + (int)L.n[a];
        }
    }
    const int NX = (int)L.N[0], NZ = (int)L.N[2];
    const dpmlk::Box3 by{0, NX, bb[1], bb[1] + L.M[1] + 1, 0, NZ};
    const dpmlk::Box3 bz{0, NX, in0[1], in1[1], bb[2], bb[2] + L.M[2] + 1};
    const dpmlk::Box3 bx{bb[0], bb[0] + L.M[0] + 1, in0[1], in1[1], in0[2], in1[2]};
    const dpmlk::Box3 bc{in0[0], in1[0], in0[1], in1[1], in0[2], in1[2]};
    const dpmlk::Box3 none{0, 0, 0, 0, 0, 0};
    dpmlk::MPlan frame{}, core{};
    frame.b[0] = make_mbox(L.M[1] > 0 ? by : none, 1, s.lchunk);
    frame.b[1] = make_mbox(L.M[2] > 0 ? bz : none, s.ryl, s.lchunk);
    frame.b[2] = make_mbox(L.M[0] > 0 ? bx : none, s.ryl, s.lchunk);
    frame.b[3] = make_mbox(none, s.ry, s.chunk);
    const bool layers = L.M[0] > 0 || L.M[1] > 0 || L.M[2] > 0;
    // algorithmic bytes: the core's cells carry no layer terms, the layer
    // boxes hold every other cell and all layer axis-cells
    double fbytes = 0, cbytes = 0;
    if (H->timing) {
        cbytes = step_bytes(H, box_cells(bc), 0.0);
        fbytes = step_bytes(H, (double)L.ncell, aux_cells(L)) - cbytes;
    }
    if (!s.split || !layers) {
        dpmlk::MPlan all = frame;
        all.b[3] = make_mbox(bc, s.ry, s.chunk);
        const int rc = launch_plan<T>(H, p, all, s, H->stream, DPML_KERNEL_STEP, fbytes + cbytes);
        if (rc) return rc;
        HIP_TRY(H, hipGetLastError());
        return DPML_OK;
    }
    core.b[0] = core.b[1] = core.b[2] = make_mbox(none, 1, 1);
    core.b[3] = make_mbox(bc, s.ry, s.chunk);
    int rc = ensure_side(H);
    if (rc) return rc;
    HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
    HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
    rc = launch_plan<T>(H, p, frame, s, H->side, DPML_KERNEL_FRAME, fbytes);
    if (!rc) rc = launch_plan<T>(H, p, core, s, H->stream, DPML_KERNEL_CORE, cbytes);
    if (rc) return rc;
    HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
    HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}

template <typename T>
int launch_march3d(dpml *H, dpmlk::StepArgs<T> p, int ry)
{
    const Layout &L = H->L;
    // periodic grids: the register-neighbour march (MARCH); walls and MARCH1
    // take the box kernels below
    if (ry != 2 && !L.wall[0] && !L.wall[1] && !L.wall[2]) return launch_mstep3d<T>(H, p, mshape(H->tile_rows));
    int b[4];
    march_box3d(L, b);
    const int NX = (int)L.N[0], NZ = (int)L.N[2];
    const bool layers = L.M[0] > 0 || L.M[1] > 0 || L.M[2] > 0;
    if (layers) {
        int rc = ensure_side(H);
        if (rc) return rc;
        HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
        HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
    }
    hipStream_t ls = layers ? H->side : H->stream;     // stream of the layer parts
    int x0 = 0, x1 = NX;
    if (L.M[0] > 0) {
        const int s0 = (L.lo[0] + 1 + 63) / 64;
        int s1 = (int)((L.lo[0] + L.n[0]) / 64);
        if (s1 < s0) s1 = s0;
        x0 = 64 * s0;
        x1 = std::min(64 * s1, NX);
    }
    const int zc = (H->tile_rows & 0xFFF) > 0 ? (H->tile_rows & 0xFFF) : 32;
    const int zl = std::max(8, zc / 4);               // layer boxes: few tiles, shorter chunks
    int rc;
    if (L.M[1] > 0) {
        const int yb = L.lo[1] + (int)L.n[1];
        rc = launch_box<T>(H, p, dpmlk::Box3{0, NX, yb, yb + L.M[1] + 1, 0, NZ}, 7, ls, DPML_KERNEL_FRAME);
        if (rc) return rc;
    }
    if (L.M[2] > 0) {
        const int zb = L.lo[2] + (int)L.n[2];
        rc = launch_box<T>(H, p, dpmlk::Box3{0, NX, b[0], b[1], zb, zb + L.M[2] + 1}, 5, ls, DPML_KERNEL_FRAME);
        if (rc) return rc;
    }
    const bool whole = !layers;
    rc = launch_zmarch<T>(H, p, dpmlk::Box3{x0, x1, b[0], b[1], b[2], b[3]}, ry, 0, zc, H->stream,
                          whole ? DPML_KERNEL_STEP : DPML_KERNEL_CORE);
    if (rc) return rc;
    if (L.M[0] > 0) {
        rc = launch_zmarch<T>(H, p, dpmlk::Box3{x1, x0 + NX, b[0], b[1], b[2], b[3]}, ry, 1, zl, ls,
                              DPML_KERNEL_FRAME);
        if (rc) return rc;
    }
    if (layers) {
        HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
        HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
    }
    HIP_TRY(H, hipGetLastError());
    return DPML_OK;
}

// Core box of a 3D two-step pass shrunk by `shrink` cells: [lo+2+shrink,
// lo+n-1-shrink) along an axis with a layer (the cells whose one-cell halo is
// free of damping terms), the whole periodic axis without one.
static dpmlk::Box3 core_box3d(const Layout &L, int shrink)
{
    int r[6];
    for (int a = 0; a < 3; ++a) {
        if (L.M[a] == 0) {
            r[2 * a] = 0;
            r[2 * a + 1] = (int)L.N[a];
            continue;
        }
        const int b0 = L.lo[a] + 2 + shrink, b1 = (int)(L.lo[a] + L.n[a]) - 1 - shrink;
        r[2 * a] = b0;
        r[2 * a + 1] = std::max(b0, b1);
    }
    return dpmlk::Box3{r[0], r[1], r[2], r[3], r[4], r[5]};
}

// 3D: two levels per pass for the multi-step variants on
// single-member grids with a constant c^2 (walls as walls_allow_multistep
// admits), planes below 4 GiB, at most 32 sources, all inside the core shrunk
// by one (the frame's steps then add none); otherwise 1.
int multistep_levels3d(const dpml *H, int64_t nsteps)
{
    const Layout &L = H->L;
    if (pass_depth(H->variant, H->tile_rows) < 2) return 1;
    if (nsteps < 2 || L.batch != 1 || H->c2_field || !walls_allow_multistep(L)) return 1;
    if (L.N[0] < 8 || L.N[1] < 8 || L.N[2] < 8 || H->ns > 32) return 1;
    // the core addresses a plane by 32-bit byte offsets
    if ((double)L.N[0] * (double)L.N[1] * (double)L.esize >= 4294967296.0) return 1;
    const dpmlk::Box3 c = core_box3d(L, 0), in1 = core_box3d(L, 1);
    if (in1.xe <= in1.xs || in1.ye <= in1.ys || in1.ze <= in1.zs) return 1;
    (void)c;
    for (int64_t cell : H->src_sorted) {
        const int x = (int)(cell % L.N[0]), y = (int)((cell / L.N[0]) % L.N[1]), z = (int)(cell / (L.N[0] * L.N[1]));
        if (x < in1.xs || x >= in1.xe || y < in1.ys || y >= in1.ye || z < in1.zs || z >= in1.ze) return 1;
    }
    return 2;
}

// One step over everything outside the box S (a frame step of a 3D pass)
// as one k_march3d_plan launch of three boxes: the rows outside S (every
// column and plane; all layer code), S's rows on the planes outside S (every
// column; x and z layer code) and S's rows and planes on the columns outside
// S (x layer code).  `bytes` is the algorithmic byte count it reports.
template <typename T>
static int launch_outside3d(dpml *H, const dpmlk::StepArgs<T> &p, const dpmlk::Box3 &S, double bytes,
                            hipStream_t st, const MShape &sh)
{
    const Layout &L = H->L;
    const int NX = (int)L.N[0], NY = (int)L.N[1], NZ = (int)L.N[2];
    const dpmlk::Box3 by{0, NX, S.ye, S.ys + NY, 0, NZ};
    const dpmlk::Box3 bz{0, NX, S.ys, S.ye, S.ze, S.zs + NZ};
    const dpmlk::Box3 bx{S.xe, S.xs + NX, S.ys, S.ye, S.zs, S.ze};
    const dpmlk::Box3 none{0, 0, 0, 0, 0, 0};
    dpmlk::MPlan pl{};
    pl.b[0] = make_mbox(S.ye - S.ys < NY ? by : none, 1, sh.lchunk);
    pl.b[1] = make_mbox(S.ze - S.zs < NZ ? bz : none, sh.ryl, sh.lchunk);
    pl.b[2] = make_mbox(S.xe - S.xs < NX ? bx : none, sh.ryl, sh.lchunk);
    pl.b[3] = make_mbox(none, 4, 1);
    MShape fs = sh;
    fs.ry = 4;
    return launch_plan<T>(H, p, pl, fs, st, DPML_KERNEL_FRAME, bytes);
}

// One step over everything outside the box S (a frame step of a 3D pass) by
// the box kernels:
// the rows outside S (every column and plane; all layer code), S's rows on
// the planes outside S (every column; x and z layer code) and S's rows and
// planes on the columns outside S (the x-band march).  `share` is the
// algorithmic byte count the three launches report together.
template <typename T>
static int launch_outside3d_boxes(dpml *H, const dpmlk::StepArgs<T> &p, const dpmlk::Box3 &S, double share,
                                  hipStream_t st)
{
    const Layout &L = H->L;
    const int NX = (int)L.N[0], NY = (int)L.N[1], NZ = (int)L.N[2];
    const dpmlk::Box3 by{0, NX, S.ye, S.ys + NY, 0, NZ};
    const dpmlk::Box3 bz{0, NX, S.ys, S.ye, S.ze, S.zs + NZ};
    const dpmlk::Box3 bx{S.xe, S.xs + NX, S.ys, S.ye, S.zs, S.ze};
    const bool hy = S.ye - S.ys < NY, hz = S.ze - S.zs < NZ, hx = S.xe - S.xs < NX;
    // each launch reports its part of the share, by its own algorithmic bytes
    double w[3] = {0, 0, 0};
    if (H->timing) {
        if (hy) w[0] = step_bytes(H, box_cells(by), box_aux(L, by));
        if (hz) w[1] = step_bytes(H, box_cells(bz), box_aux(L, bz));
        if (hx) w[2] = step_bytes(H, box_cells(bx), box_aux(L, bx));
        const double sum = w[0] + w[1] + w[2];
        for (double &v : w) v = sum > 0 ? share * v / sum : 0;
    }
    int rc = DPML_OK;
    if (hy) rc = launch_box<T>(H, p, by, 7, st, DPML_KERNEL_FRAME, w[0]);
    if (rc) return rc;
    if (hz) rc = launch_box<T>(H, p, bz, 5, st, DPML_KERNEL_FRAME, w[1]);
    if (rc) return rc;
    if (hx) {
        const int zc = (H->tile_rows & 0xFFF) > 0 ? (H->tile_rows & 0xFFF) : 32;
        rc = launch_zmarch<T>(H, p, bx, 4, 1, std::max(8, zc / 4), st, DPML_KERNEL_FRAME, w[2]);
    }
    return rc;
}

// Two steps of a 3D grid.  The core kernel runs on the handle's stream; the
// frame takes two ordinary steps on the side stream at the same time, step
// j over everything outside the core shrunk by 2 - j cells.  The core writes
// U^{n+1} only on the core shrunk by one, so every cell of every buffer has
// one writer.  With bit 30 of tile_rows (periodic axes) the frame instead
// takes both levels in one march per box (launch_frame2_3d) over everything
// outside the core, which then writes U^{n+1} on the whole core; that frame
// reads the aux buffer of level n and writes level n+2 to the other one, so
// the pass flips the aux index.  Receivers and the plane record both levels
// once the side stream has joined.
template <typename T>
int launch_multistep3d(dpml *H)
{
    const Layout &L = H->L;
    T *A = (T *)H->u_now, *Bv = (T *)H->u_old;
    T *nxt[2] = {nullptr, nullptr};
    int k = 0;
    for (int i = 0; i < L.n_ubuf && k < 2; ++i) {
        void *b = H->at(L.off_u[i]);
        if (b != H->u_now && b != H->u_old) nxt[k++] = (T *)b;
    }
    if (k < 2) return H->fail(DPML_EINVAL, "not enough field buffers for a multi-step pass");
    // the marching frames (bits 19 and 30) take periodic axes only; bits
    // 18-29 describe the two-level frame when bit 30 is set
    const bool periodic = !L.wall[0] && !L.wall[1] && !L.wall[2];
    const bool f2bit = (H->tile_rows >> 30) & 1;
    const bool frame2 = f2bit && periodic;
    const dpmlk::Box3 c = core_box3d(L, 0), in1 = frame2 ? c : core_box3d(L, 1);
    // tile_rows: planes per chunk in the low 12 bits (0: 32), rows per wave
    // in bits 12-17 (4, 8 or 16; 0: 8); the frame's steps by the
    // register-neighbour march when bit 19 is set on a periodic grid (planes
    // per layer chunk in bits 20-27, as in mshape), else by the box kernels;
    // bit 28 the core's tiles in launch order; bit 29 below
    const int chunk = (H->tile_rows & 0xFFF) > 0 ? (H->tile_rows & 0xFFF) : 32;
    const int ryb = (H->tile_rows >> 12) & 0x3F;
    const int ry = (ryb == 4 || ryb == 16) ? ryb : 8;
    const MShape fsh = mshape(H->tile_rows & ~0xFFFF);
    const int ord = (H->tile_rows >> 28) & 1;
    const bool frame_plan = !f2bit && periodic && ((H->tile_rows >> 19) & 1);
    // bit 29: the frame's first step alone on the handle's stream first, then
    // the core beside the frame's second step (else the core beside both)
    const bool frame_first = !f2bit && ((H->tile_rows >> 29) & 1);
    // the frame's step j (1 or 2) on stream st, aux buffers alternating
    auto frame_step = [&](int j, hipStream_t st) -> int {
        if (j == 2) H->cur = 1 - H->cur;
        dpmlk::StepArgs<T> pj = make_args<T>(H);
        if (j == 2) H->cur = 1 - H->cur;
        pj.u = j == 1 ? A : nxt[0];
        pj.uo = j == 1 ? Bv : A;
        pj.uout = nxt[j - 1];
        // algorithmic share: the frame's own cells (the ring cells it recomputes
        // are the core's, counted there)
        const double share = step_bytes(H, (double)L.ncell - box_cells(c), aux_cells(L));
        return frame_plan ? launch_outside3d<T>(H, pj, core_box3d(L, 2 - j), share, st, fsh)
                          : launch_outside3d_boxes<T>(H, pj, core_box3d(L, 2 - j), share, st);
    };
    if (frame_first) {
        int rc = frame_step(1, H->stream);
        if (rc) return rc;
    }
    HIP_TRY(H, hipEventRecord(H->ev_fork, H->stream));
    HIP_TRY(H, hipStreamWaitEvent(H->side, H->ev_fork, 0));
    {
        dpmlk::StepArgs<T> p = make_args<T>(H);
        p.uout = nxt[0];
        p.tile_rows = chunk;
        p.tiles_x = (c.xe - c.xs + 59) / 60;
        p.tiles_y = (c.ye - c.ys + 4 * ry - 1) / (4 * ry);
        p.n_tiles = p.tiles_x * p.tiles_y * ((c.ze - c.zs + chunk - 1) / chunk);
        dpmlk::Src3<T> src{};
        src.cells = H->d_src_cells;
        src.order = H->d_src_order;
        src.wav = (const T *)H->wavelets;
        src.ns = H->ns;
        src.nt = H->nt_src;
        src.n = H->n;
        src.amp = (T)(H->dt * H->dt / (H->h * H->h * H->h));
        const double core = box_cells(c);
        const int slot = timed_begin(H, DPML_KERNEL_PAIR, pass_bytes(H, core));
        const dim3 grid((unsigned)round8(p.n_tiles)), block(256);
#define DPML_TWO3D(RY_, O_) \
    hipLaunchKernelGGL((dpmlk::k_step2_zmarch3d<T, RY_, O_>), grid, block, 0, H->stream, p, nxt[1], c, in1, src)
        if (ry == 4) {
            if (ord) DPML_TWO3D(4, 1); else DPML_TWO3D(4, 0);
        } else if (ry == 16) {
            if (ord) DPML_TWO3D(16, 1); else DPML_TWO3D(16, 0);
        } else {
            if (ord) DPML_TWO3D(8, 1); else DPML_TWO3D(8, 0);
        }
#undef DPML_TWO3D
        timed_end(H, slot);
    }
    if (frame2) {
        // both levels of the frame in one march per box, beside the core
        const dpmlk::StepArgs<T> pf = make_args<T>(H);
        int rc = launch_frame2_3d<T>(H, pf, nxt[0], nxt[1], c, H->tile_rows, H->side, H->stream);
        if (rc) return rc;
        H->cur = 1 - H->cur;
    } else {
        // the frame's (remaining) steps on the side stream beside the core
        for (int j = frame_first ? 2 : 1; j <= 2; ++j) {
            int rc = frame_step(j, H->side);
            if (rc) return rc;
        }
    }
    HIP_TRY(H, hipEventRecord(H->ev_join, H->side));
    HIP_TRY(H, hipStreamWaitEvent(H->stream, H->ev_join, 0));
    HIP_TRY(H, hipGetLastError());
    int rc = launch_record<T>(H, nxt[0], H->n);
    if (rc) return rc;
    rc = launch_record<T>(H, nxt[1], H->n + 1);
    if (rc) return rc;
    H->u_now = nxt[1];
    H->u_old = nxt[0];
    H->n += 2;
    return DPML_OK;
}

template int launch_march3d<float>(dpml *, dpmlk::StepArgs<float>, int);
template int launch_march3d<double>(dpml *, dpmlk::StepArgs<double>, int);
template int launch_multistep3d<float>(dpml *);
template int launch_multistep3d<double>(dpml *);

}  // namespace dpmlh
