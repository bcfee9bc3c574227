"""Test glue: move states between the GPU binding and the oracle, and
compare fields the way the parity tolerances are stated (max abs error over
the field divided by the field's peak in the oracle)."""
import numpy as np

import oracle


def band_indices(n, lo, hi):
    """Array index of band slot j = 0..M along one axis."""
    N = lo + n + hi
    M = lo + hi
    return [(lo + n + j) % N for j in range(M + 1)]


def expand_aux(compact: np.ndarray, axis: int, n, lo, hi, kind: str) -> np.ndarray:
    """Embed a compact band array (numpy shape reversed, x last) into a full
    field, writing only the slots where the auxiliary is defined
    (Phi: j in [0, M-1], Psi: j in [1, M])."""
    d = compact.ndim
    N = [lo[a] + n[a] + hi[a] for a in range(d)]
    full = np.zeros(tuple(reversed(N)))
    M = lo[axis] + hi[axis]
    idx = band_indices(n[axis], lo[axis], hi[axis])
    js = range(0, M) if kind == "phi" else range(1, M + 1)
    npax = d - 1 - axis
    for j in js:
        src = [slice(None)] * d
        dst = [slice(None)] * d
        src[npax] = j
        dst[npax] = idx[j]
        full[tuple(dst)] = compact[tuple(src)]
    return full


def support_mask(axis: int, n, lo, hi, kind: str) -> np.ndarray:
    d = len(n)
    N = [lo[a] + n[a] + hi[a] for a in range(d)]
    m1 = np.zeros(N[axis], dtype=bool)
    M = lo[axis] + hi[axis]
    idx = band_indices(n[axis], lo[axis], hi[axis])
    js = range(0, M) if kind == "phi" else range(1, M + 1)
    for j in js:
        m1[idx[j]] = True
    shape = [1] * d
    shape[d - 1 - axis] = N[axis]
    return np.broadcast_to(m1.reshape(shape), tuple(reversed(N)))


def gpu_state(sim):
    """Download a Simulation's current level as an oracle.State (FP64)."""
    import paper_1804_01390_amd as dp
    sim.sync()
    U = sim.field(dp.FIELD_U).double().cpu().numpy()
    Up = sim.field(dp.FIELD_UPREV).double().cpu().numpy()
    Phi, Psi = [], []
    for a in range(sim.ndim):
        if sim.lo[a] + sim.hi[a] == 0:
            Phi.append(np.zeros_like(U))
            Psi.append(np.zeros_like(U))
            continue
        Phi.append(expand_aux(sim.field(dp.FIELD_PHI(a)).double().cpu().numpy(), a, sim.n, sim.lo, sim.hi, "phi"))
        Psi.append(expand_aux(sim.field(dp.FIELD_PSI(a)).double().cpu().numpy(), a, sim.n, sim.lo, sim.hi, "psi"))
    return oracle.State(U, Up, Phi, Psi, sim.time_index)


def multi_state(sim, prob: int, w):
    """Download problem ``prob`` of a MultiSimulation (workload ``w``) as an
    oracle.State (FP64)."""
    import paper_1804_01390_amd as dp
    sim.sync()
    U = sim.field(prob, dp.FIELD_U).double().cpu().numpy()
    Up = sim.field(prob, dp.FIELD_UPREV).double().cpu().numpy()
    Phi = [expand_aux(sim.field(prob, dp.FIELD_PHI(a)).double().cpu().numpy(), a, w.n, w.lo, w.hi, "phi")
           for a in range(2)]
    Psi = [expand_aux(sim.field(prob, dp.FIELD_PSI(a)).double().cpu().numpy(), a, w.n, w.lo, w.hi, "psi")
           for a in range(2)]
    return oracle.State(U, Up, Phi, Psi, 0)


def rel_err(got, ref, mask=None) -> float:
    if mask is not None:
        got = got[mask]
        ref = ref[mask]
    peak = float(np.max(np.abs(ref))) if ref.size else 0.0
    if peak == 0.0:
        return float(np.max(np.abs(got))) if got.size else 0.0
    return float(np.max(np.abs(got - ref)) / peak)


def compare_states(gs, os_, n, lo, hi, peaks=None):
    """Per-field normalised max errors: U, Uprev, Phi_a/Psi_a on their
    supports.  Normalised by the oracle field's peak at the compared step, or,
    when ``peaks`` is given, by the field's peak over the whole run (see
    run_peaks) -- the FP32 reading: FP32 rounding scales with the largest
    values a run has carried, not with what is left after the layer has
    absorbed most of the wave."""
    def e(key, got, ref, mask=None):
        if peaks is None:
            return rel_err(got, ref, mask)
        g = got[mask] if mask is not None else got
        r = ref[mask] if mask is not None else ref
        return float(np.max(np.abs(g - r))) / peaks[key] if r.size else 0.0

    errs = {"U": e("U", gs.U, os_.U), "Uprev": e("U", gs.Uprev, os_.Uprev)}
    for a in range(len(n)):
        if lo[a] + hi[a] == 0:
            continue
        errs["Phi%d" % a] = e("Phi%d" % a, gs.Phi[a], os_.Phi[a], support_mask(a, n, lo, hi, "phi"))
        errs["Psi%d" % a] = e("Psi%d" % a, gs.Psi[a], os_.Psi[a], support_mask(a, n, lo, hi, "psi"))
    return errs


def run_with_peaks(g, state, steps, n, lo, hi, chunks=10, **kw):
    """Run the oracle in chunks and return (final state, traces, peaks) where
    peaks[field] is the field's max magnitude over the run (U over the whole
    grid, Phi_a/Psi_a over their supports), sampled at chunk ends."""
    peaks = {}

    def upd(s):
        peaks["U"] = max(peaks.get("U", 0.0), float(np.max(np.abs(s.U))), float(np.max(np.abs(s.Uprev))))
        for a in range(len(n)):
            if lo[a] + hi[a] == 0:
                continue
            for kind, arr in (("Phi", s.Phi[a]), ("Psi", s.Psi[a])):
                m = support_mask(a, n, lo, hi, kind.lower())
                key = "%s%d" % (kind, a)
                peaks[key] = max(peaks.get(key, 0.0), float(np.max(np.abs(arr[m]))))

    kw.setdefault("nt", state.n + steps)
    upd(state)
    done = 0
    traces = None
    step = max(1, steps // chunks)
    while done < steps:
        k = min(step, steps - done)
        state, tr = oracle.run(g, state, k, **kw)
        traces = tr if traces is None else traces + tr   # each chunk fills its own columns
        done += k
        upd(state)
    for key in list(peaks):
        if peaks[key] == 0.0:
            peaks[key] = 1.0
    # an auxiliary field that never rises above FP32's rounding of the run's
    # largest U values (a layer the wave has not reached: ~1e-200 in FP64,
    # underflowing to 0 in FP32) is measured on the scale of that rounding
    for key in list(peaks):
        if key != "U":
            peaks[key] = max(peaks[key], peaks["U"] * 2.0 ** -24)
    return state, traces, peaks
