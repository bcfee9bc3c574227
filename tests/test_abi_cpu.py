"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid configurations before touching the GPU
(validation happens on the host, so no device is needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1804_01390_amd as dp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dpml.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpml_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = dp.load_library()
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(dp.EXPORTED) == names


def test_header_parses_as_c():
    import subprocess
    r = subprocess.run(["gcc", "-fsyntax-only", "-Wall", "-Werror", "-x", "c", "-std=c99", "-"],
                       input='#include "dpml.h"\nint main(void){return 0;}\n', text=True,
                       capture_output=True, cwd=os.path.join(ROOT, "include"))
    assert r.returncode == 0, r.stderr


def _defines():
    src = open(os.path.join(ROOT, "include", "dpml.h")).read()
    return {m.group(1): int(m.group(2)) for m in
            re.finditer(r"#define (DPML_[A-Z0-9_]+) \(?(-?\d+)\)?", src)}


def test_binding_constants_match_the_header():
    d = _defines()
    assert len(d) >= 20
    for name, value in d.items():
        py = name[len("DPML_"):] if name.startswith(("DPML_VARIANT_", "DPML_KERNEL_", "DPML_FIELD_", "DPML_PROBE_")) else name
        assert getattr(dp, py) == value, name
    for a in range(3):
        assert dp.FIELD_PHI(a) == 2 + 2 * a and dp.FIELD_PSI(a) == 3 + 2 * a


def test_tuner_candidates_are_valid_launch_shapes():
    """Every shape the tuner may apply lies inside the ranges dpml_set_variant
    and dpml_multi_set_variant accept (depth 2..8 for DEEP, load group 1, 2
    or 4, frame form 0..15, rows within the kernels' limits)."""
    from paper_1804_01390_amd import autotune
    multi_variants = (dp.VARIANT_TWOSTEP, dp.VARIANT_THREESTEP, dp.VARIANT_FOURSTEP, dp.VARIANT_DEEP)
    for variant, tr in autotune.CANDIDATES_2D:
        assert dp.VARIANT_AUTO <= variant <= dp.VARIANT_DEEP
        assert 0 <= tr < (1 << (25 if variant == dp.VARIANT_DEEP else 20))
    for variant, tr in autotune.CANDIDATES_3D:       # 3D MARCH shapes take bits up to 29, passes up to 30
        assert dp.VARIANT_AUTO <= variant <= dp.VARIANT_DEEP
        top = 20 if variant in (dp.VARIANT_CELL, dp.VARIANT_MARCH1) else (30 if variant == dp.VARIANT_MARCH else 31)
        assert 0 <= tr < (1 << (25 if variant == dp.VARIANT_DEEP else top))
        if variant == dp.VARIANT_DEEP:
            assert ((tr >> 20) & 0xF) in (0, 2, 3, 4, 5, 6, 7, 8)
    for variant, tr in autotune.CANDIDATES_2D:
        if variant in multi_variants:
            assert ((tr >> 12) & 0xF) in (0, 1, 2, 4) and 0 < (tr & 0xFFF) <= 4095
    for variant, tr in autotune.CANDIDATES_3D:
        if variant in multi_variants:          # 3D passes: rows per wave in bits 12-17, planes per chunk below
            assert ((tr >> 12) & 0x3F) in (4, 8, 16) and 0 < (tr & 0xFFF) <= 4095
        if variant == dp.VARIANT_MARCH:        # marching steps: rows per core wave in bits 12-15
            assert ((tr >> 12) & 0xF) in (1, 2, 4, 8) and ((tr >> 16) & 3) in (0, 1, 2)
            assert (tr & 0xFFF) > 0 and ((tr >> 20) & 0xFF) > 0
    for variant, rows, group in autotune.CANDIDATES_MULTI:
        assert variant in (dp.VARIANT_MARCH,) + multi_variants
        assert group in (1, 2, 4)
        if variant == dp.VARIANT_DEEP:
            assert ((rows >> 20) & 0xF) in (2, 3, 4, 5, 6, 7, 8) and 1 <= (rows & 0xFFFFF) <= 4096
        else:
            assert (4 if variant == dp.VARIANT_MARCH else 1) <= rows <= 4096


def test_pass_shape_packs_the_documented_bits():
    assert dp.pass_shape() == 0
    assert dp.pass_shape(rows=32, group=4, depth=8, ahead=True) == (1 << 24) | (8 << 20) | (4 << 12) | 32
    assert dp.pass_shape(rows=6, frame=15, depth=6) == (6 << 20) | (15 << 16) | 6
    for bad in (dict(rows=4096), dict(group=3), dict(frame=16), dict(depth=1), dict(depth=9)):
        with pytest.raises(ValueError):
            dp.pass_shape(**bad)


def test_workspace_holds_the_multistep_buffers():
    """2D handles carry U^n, U^{n-1} and eight more U arrays (passes of up to
    eight levels write U^{n+1} .. U^{n+8}); 3D handles two more."""
    lib = dp.load_library()
    for ndim, n, esize, ubufs in [(2, [100, 80], 4, 10), (3, [20, 18, 16], 8, 4)]:
        g = dp._grid(n, [0] * ndim, [0] * ndim, dp.DPML_F32 if esize == 4 else dp.DPML_F64)
        cells = int(np.prod(n))
        assert lib.dpml_workspace_bytes(ctypes.byref(g), 0) >= ubufs * cells * esize


def _create(n, lo, hi, h=1.0, dt=0.5, sigma=None, c2=(1.0,), dtype=dp.DPML_F64, ws_bytes=None,
            ws_ptr=4096):
    lib = dp.load_library()
    g = dp._grid(n, lo, hi, dtype)
    c2a = np.ascontiguousarray(np.asarray(c2, dtype=np.float64).reshape(-1))
    sig3 = (dp._DP * 3)()
    keep = []
    for a in range(3):
        if sigma is not None and a < len(sigma) and sigma[a] is not None:
            s = np.ascontiguousarray(sigma[a], dtype=np.float64)
            keep.append(s)
            sig3[a] = s.ctypes.data_as(dp._DP)
        else:
            sig3[a] = dp._DP()
    need = lib.dpml_workspace_bytes(ctypes.byref(g), 1 if c2a.size != 1 else 0)
    out = dp._VP()
    rc = lib.dpml_create(ctypes.byref(g), h, dt, c2a.ctypes.data_as(dp._DP), c2a.size, sig3,
                         ctypes.c_void_p(ws_ptr), need if ws_bytes is None else ws_bytes, None,
                         ctypes.byref(out))
    return rc, lib.dpml_last_error(None).decode(), need


def _ramp(n, lo, hi, smax=2.0):
    import synthetic
    return synthetic.sigma_ramp(n, lo, hi, smax)


def test_workspace_bytes_accounts_for_fields():
    lib = dp.load_library()
    g = dp._grid([100, 80], [8, 8], [8, 8], dp.DPML_F32)
    b0 = lib.dpml_workspace_bytes(ctypes.byref(g), 0)
    b1 = lib.dpml_workspace_bytes(ctypes.byref(g), 1)
    N = 116 * 96
    assert b0 >= 2 * N * 4 + 2 * 2 * (17 * 96 + 116 * 17) * 4
    assert b1 - b0 >= N * 4
    bad = dp._grid([100, 80], [8, 8], [8, 8], 7)
    assert lib.dpml_workspace_bytes(ctypes.byref(bad), 0) == 0


@pytest.mark.parametrize("case,code", [
    ("cfl", dp.DPML_EINVAL),
    ("neg_sigma", dp.DPML_EINVAL),
    ("sigma_in_interior", dp.DPML_EINVAL),
    ("nan_sigma", dp.DPML_EINVAL),
    ("dt_sigma", dp.DPML_EINVAL),
    ("c2_in_layer", dp.DPML_EINVAL),
    ("c2_const_not_one", dp.DPML_EINVAL),
    ("c2_bad_len", dp.DPML_EINVAL),
    ("ndim", dp.DPML_EINVAL),
    ("ws_small", dp.DPML_ENOMEM),
    ("ws_misaligned", dp.DPML_ENOMEM),
    ("h_zero", dp.DPML_EINVAL),
])
def test_create_rejects_invalid_configurations(case, code):
    n, lo, hi = [32, 24], [4, 4], [4, 4]
    sig = [_ramp(32, 4, 4), _ramp(24, 4, 4)]
    kw = {}
    if case == "cfl":
        kw["dt"] = 0.75          # 0.75 * sqrt(2) > 1
    elif case == "neg_sigma":
        sig[0] = sig[0].copy(); sig[0][0] = -1.0
    elif case == "sigma_in_interior":
        sig[1] = sig[1].copy(); sig[1][10] = 0.5
    elif case == "nan_sigma":
        sig[0] = sig[0].copy(); sig[0][1] = np.nan
    elif case == "dt_sigma":
        sig[0] = sig[0] * 10.0   # dt * sigma_max = 0.5 * 15.3 > 4
    elif case == "c2_in_layer":
        c2 = np.ones((32, 40)); c2[1, 20] = 1.2
        kw["c2"] = c2
    elif case == "c2_const_not_one":
        kw["c2"] = (0.8,)
    elif case == "c2_bad_len":
        kw["c2"] = np.ones(17)
    elif case == "ndim":
        n, lo, hi = [32], [4], [4]
    elif case == "ws_small":
        kw["ws_bytes"] = 1024
    elif case == "ws_misaligned":
        kw["ws_ptr"] = 4096 + 8
    elif case == "h_zero":
        kw["h"] = 0.0
    rc, msg, _ = _create(n, lo, hi, sigma=sig, **kw)
    assert rc == code, (rc, msg)
    assert msg


def test_c2_field_allowed_away_from_layer_validates():
    """A c^2 field that is 1 on and next to the layer passes validation (the
    call then fails only when it reaches the GPU, which this box lacks)."""
    n, lo, hi = [32, 24], [4, 4], [4, 4]
    c2 = np.ones((32, 40)); c2[16, 20] = 1.3
    rc, msg, _ = _create(n, lo, hi, sigma=[_ramp(32, 4, 4), _ramp(24, 4, 4)], c2=c2, dt=0.4)
    assert rc in (dp.DPML_OK, dp.DPML_EHIP), msg
    assert "c2" not in msg


def test_strerror_covers_codes():
    lib = dp.load_library()
    for c in (0, -1, -2, -3, -4, -5):
        assert lib.dpml_strerror(c).decode() not in ("", "unknown error")
    assert lib.dpml_strerror(-99).decode() == "unknown error"


def test_null_handle_calls_are_rejected():
    lib = dp.load_library()
    assert lib.dpml_step(None, 1) == dp.DPML_EINVAL
    assert lib.dpml_sync(None) == dp.DPML_EINVAL
    assert lib.dpml_time_index(None) == -1
    lib.dpml_destroy(None)


def test_package_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        dp.Simulation([16, 16], [2, 2], [2, 2], 1.0, 0.5, [None, None])
