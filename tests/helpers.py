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


def rel_err(got, ref, mask=None) -> float:
    if mask is not None:
        got = got[mask]
        ref = ref[mask]
    peak = float(np.max(np.abs(ref))) if ref.size else 0.0
    if peak == 0.0:
        return float(np.max(np.abs(got))) if got.size else 0.0
    return float(np.max(np.abs(got - ref)) / peak)


def compare_states(gs, os_, n, lo, hi):
    """Per-field peak-normalised errors: U, Uprev, Phi_a/Psi_a on their supports."""
    errs = {"U": rel_err(gs.U, os_.U), "Uprev": rel_err(gs.Uprev, os_.Uprev)}
    for a in range(len(n)):
        if lo[a] + hi[a] == 0:
            continue
        errs["Phi%d" % a] = rel_err(gs.Phi[a], os_.Phi[a], support_mask(a, n, lo, hi, "phi"))
        errs["Psi%d" % a] = rel_err(gs.Psi[a], os_.Psi[a], support_mask(a, n, lo, hi, "psi"))
    return errs
