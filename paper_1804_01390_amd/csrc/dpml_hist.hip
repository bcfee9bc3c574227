// dpml_hist.hip -- the 2D multi-step pass that keeps every level it forms
// (the recompute of the checkpointed adjoint: each U^k of a segment is
// needed once by the reverse sweep).  The arithmetic is that of the ordinary
// pass, Eq. (DiscretePML a) of Chern, "A Reflectionless Discrete Perfectly
// Matched Layer", on the layer-free core; only the stores differ.
#include "dpml_host.hpp"

namespace dpmlh {

template <typename T, int VX, int G, bool C2>
static void launch_hist_g(int levels, dim3 grid, hipStream_t st, const dpmlk::StepArgs<T> &p, T *hist,
                          int64_t hstride, T *pen, T *fin, const int r[4], int strips, int n_waves,
                          const dpmlk::Taps2<T> &tp)
{
    const dim3 block(256);
#define DPML_HIST_N(NL)                                                                                      \
    hipLaunchKernelGGL((dpmlk::k_stepN_hist<T, VX, G, C2, NL>), grid, block, 0, st, p, hist, hstride, pen, fin, \
                       r[0], r[1], r[2], r[3], strips, n_waves, tp)
    switch (levels) {
    case 4: DPML_HIST_N(4); break;
    case 5: DPML_HIST_N(5); break;
    case 6: DPML_HIST_N(6); break;
    case 7: DPML_HIST_N(7); break;
    default: DPML_HIST_N(8); break;
    }
#undef DPML_HIST_N
}

template <typename T>
void launch_coreN_hist(int levels, int G, bool c2, dim3 grid, hipStream_t st, const dpmlk::StepArgs<T> &p, T *hist,
                       int64_t hstride, T *pen, T *fin, const int r[4], int strips, int n_waves,
                       const dpmlk::Taps2<T> &tp)
{
    constexpr int VX = sizeof(T) == 4 ? 4 : 2;
#define DPML_HIST_G(GG)                                                                                    \
    if (c2)                                                                                                \
        launch_hist_g<T, VX, GG, true>(levels, grid, st, p, hist, hstride, pen, fin, r, strips, n_waves, tp); \
    else                                                                                                   \
        launch_hist_g<T, VX, GG, false>(levels, grid, st, p, hist, hstride, pen, fin, r, strips, n_waves, tp)
    if (G == 4) {
        DPML_HIST_G(4);
    } else if (G == 1) {
        DPML_HIST_G(1);
    } else {
        DPML_HIST_G(2);
    }
#undef DPML_HIST_G
}

template void launch_coreN_hist<float>(int, int, bool, dim3, hipStream_t, const dpmlk::StepArgs<float> &, float *,
                                       int64_t, float *, float *, const int *, int, int,
                                       const dpmlk::Taps2<float> &);
template void launch_coreN_hist<double>(int, int, bool, dim3, hipStream_t, const dpmlk::StepArgs<double> &, double *,
                                        int64_t, double *, double *, const int *, int, int,
                                        const dpmlk::Taps2<double> &);

}  // namespace dpmlh
