// dpml_frame3d.hip -- the frame of a 3D two-step pass taken as two levels in
// one march (k_frame2_box3d): Eq. (DiscretePML a-c) of Chern, "A
// Reflectionless Discrete Perfectly Matched Layer", twice over every cell
// outside the core box, the layer auxiliaries of the middle level kept in
// registers.  Its own translation unit: 20 kernel shapes per precision.
#include "dpml_host.hpp"
#include "dpml_kernels3d.hpp"

namespace dpmlh {

// Waves of one frame box: strips of 60 output columns, groups of `ry` rows,
// chunks of at most `chunk` planes.
static dpmlk::MBox make_f2box(const dpmlk::Box3 &bx, int ry, int chunk)
{
    dpmlk::MBox m{bx.xs, bx.xe, bx.ys, bx.ye, bx.zs, bx.ze, 0, 0, 1, 0};
    if (bx.xe <= bx.xs || bx.ye <= bx.ys || bx.ze <= bx.zs) return m;   // no waves
    m.strips = (bx.xe - bx.xs + 59) / 60;
    m.groups = (bx.ye - bx.ys + ry - 1) / ry;
    m.chunk = std::max(1, std::min(chunk, bx.ze - bx.zs));
    m.chunks = (bx.ze - bx.zs + m.chunk - 1) / m.chunk;
    return m;
}

template <typename T, int RY, int AX, bool PA>
static int f2_launch(dpml *H, const dpmlk::MBox &m, hipStream_t st, const dpmlk::StepArgs<T> &p, T *out1, T *out2,
                     double bytes)
{
    const int64_t w = (int64_t)m.strips * m.groups * m.chunks;
    if (w == 0) return DPML_OK;
    if (w > ((int64_t)1 << 30)) return H->fail(DPML_EINVAL, "3D grid too large for one frame launch");
    const int slot = timed_begin(H, DPML_KERNEL_FRAME, bytes, st);
    hipLaunchKernelGGL((dpmlk::k_frame2_box3d<T, RY, AX, PA>), dim3((unsigned)round8((int)((w + 3) / 4))), dim3(256),
                       0, st, p, out1, out2, m);
    timed_end(H, slot, st);
    return DPML_OK;
}

// A box outside the core along the axes of `ax` (bit a for axis a): the
// boxes outside along one axis take `ry` rows per wave (2 or 4), the others 2.
template <typename T, bool PA>
static int f2_launch_ax(dpml *H, int ax, int ry, const dpmlk::MBox &m, hipStream_t st, const dpmlk::StepArgs<T> &p,
                        T *out1, T *out2, double bytes)
{
    switch (ax) {
    case 1: return ry == 4 ? f2_launch<T, 4, 1, PA>(H, m, st, p, out1, out2, bytes)
                           : f2_launch<T, 2, 1, PA>(H, m, st, p, out1, out2, bytes);
    case 2: return ry == 4 ? f2_launch<T, 4, 2, PA>(H, m, st, p, out1, out2, bytes)
                           : f2_launch<T, 2, 2, PA>(H, m, st, p, out1, out2, bytes);
    case 4: return ry == 4 ? f2_launch<T, 4, 4, PA>(H, m, st, p, out1, out2, bytes)
                           : f2_launch<T, 2, 4, PA>(H, m, st, p, out1, out2, bytes);
    case 3: return f2_launch<T, 2, 3, PA>(H, m, st, p, out1, out2, bytes);
    case 5: return f2_launch<T, 2, 5, PA>(H, m, st, p, out1, out2, bytes);
    case 6: return f2_launch<T, 2, 6, PA>(H, m, st, p, out1, out2, bytes);
    default: return f2_launch<T, 2, 7, PA>(H, m, st, p, out1, out2, bytes);
    }
}

template <typename T>
int launch_frame2_3d(dpml *H, const dpmlk::StepArgs<T> &p, T *out1, T *out2, const dpmlk::Box3 &c, int shape,
                     hipStream_t st, hipStream_t st2)
{
    const Layout &L = H->L;
    // shape bit 18: rows per wave of the boxes outside c along one axis (0: 2,
    // 1: 4; the others take 2); bit 20: planes per chunk of the boxes outside
    // along two or three axes (0: 8, 1: 4); bits 21-25: planes per chunk of the
    // x and y boxes, in eights (0: 32); bits 26-27: chunks of the z box (0: 1,
    // 1: 2, 2: 4, 3: 8); bit 29: the layer arrays loaded at their own plane
    // instead of a plane ahead; bit 19: the boxes outside along two or three
    // axes as one launch on st2 (else one launch each on st)
    const int ry1 = ((shape >> 18) & 1) ? 4 : 2;
    const int mchunk = ((shape >> 20) & 1) ? 4 : 8;
    const int lc = (shape >> 21) & 0x1F;
    const int lchunk = lc ? 8 * lc : 32;
    const int zparts = 1 << ((shape >> 26) & 3);
    const bool pa = !((shape >> 29) & 1);
    // per axis: c's range and the range outside it (across the periodic wrap)
    const int cs[3] = {c.xs, c.ys, c.zs}, ce[3] = {c.xe, c.ye, c.ze};
    int out1_[3];
    for (int a = 0; a < 3; ++a)
        out1_[a] = ce[a] - cs[a] < (int)L.N[a] ? cs[a] + (int)L.N[a] : ce[a];   // empty without a layer
    // the boxes outside c along one axis first (the large ones); with bit 19
    // the others as one launch on st2
    const bool edges = (shape >> 19) & 1;
    dpmlk::F2Edges eb{};
    double ebytes = 0.0;
    int64_t ew = 0;
    static const int order[7] = {1, 2, 4, 3, 5, 6, 7};
    for (int ax : order) {
        int r0[3], r1[3];
        for (int a = 0; a < 3; ++a) {
            const bool out = (ax >> a) & 1;
            r0[a] = out ? ce[a] : cs[a];
            r1[a] = out ? out1_[a] : ce[a];
        }
        const dpmlk::Box3 b{r0[0], r1[0], r0[1], r1[1], r0[2], r1[2]};
        if (b.xe <= b.xs || b.ye <= b.ys || b.ze <= b.zs) continue;
        const bool single = ax == 1 || ax == 2 || ax == 4;
        const int ry = single ? ry1 : 2;
        const int chunk = !single ? mchunk : (ax == 4 ? (b.ze - b.zs + zparts - 1) / zparts : lchunk);
        const dpmlk::MBox m = make_f2box(b, ry, chunk);
        // algorithmic bytes per pass: U^n, U^{n-1} read and two levels
        // written per cell, Phi/Psi read and written once per layer axis-cell
        const double bytes = H->timing ? (4.0 * box_cells(b) + 4.0 * box_aux(L, b)) * (double)L.esize : 0.0;
        if (edges && !single) {
            const int i = ax == 3 ? 0 : (ax == 5 ? 1 : (ax == 6 ? 2 : 3));
            eb.b[i] = m;
            ebytes += bytes;
            continue;
        }
        const int rc = pa ? f2_launch_ax<T, true>(H, ax, ry, m, st, p, out1, out2, bytes)
                          : f2_launch_ax<T, false>(H, ax, ry, m, st, p, out1, out2, bytes);
        if (rc) return rc;
    }
    if (edges) {
        for (int i = 0; i < 4; ++i) {
            ew += (int64_t)eb.b[i].strips * eb.b[i].groups * eb.b[i].chunks;   // empty boxes have no waves
            eb.w[i] = (int32_t)std::min<int64_t>(ew, (int64_t)1 << 30);
        }
        if (ew > ((int64_t)1 << 30)) return H->fail(DPML_EINVAL, "3D grid too large for one frame launch");
        if (ew > 0) {
            const int slot = timed_begin(H, DPML_KERNEL_FRAME, ebytes, st2);
            const dim3 g((unsigned)round8((int)((ew + 3) / 4))), b(256);
            if (pa) hipLaunchKernelGGL((dpmlk::k_frame2_edges3d<T, true>), g, b, 0, st2, p, out1, out2, eb);
            else hipLaunchKernelGGL((dpmlk::k_frame2_edges3d<T, false>), g, b, 0, st2, p, out1, out2, eb);
            timed_end(H, slot, st2);
        }
    }
    return DPML_OK;
}

template int launch_frame2_3d<float>(dpml *, const dpmlk::StepArgs<float> &, float *, float *, const dpmlk::Box3 &,
                                     int, hipStream_t, hipStream_t);
template int launch_frame2_3d<double>(dpml *, const dpmlk::StepArgs<double> &, double *, double *,
                                      const dpmlk::Box3 &, int, hipStream_t, hipStream_t);

}  // namespace dpmlh
