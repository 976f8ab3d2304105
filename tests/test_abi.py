"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-only calls (validation, buffer sizes) behave as the
header states.  No call here needs a GPU."""
import ctypes as C
import math
import os
import re

import pytest

import paper_2301_06061_amd as ws
from paper_2301_06061_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wstack.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ws_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ws.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in wstack.h but not exported"
    # the binding declares exactly the header's entry points
    assert sorted(_abi.exported_symbols()) == names


def _p(**kw):
    base = dict(nu=512, nv=512, nw=8, fov_l=math.radians(1), fov_m=math.radians(1),
                w_min=-100.0, w_max=100.0, support=7, sigma=0.0,
                precision="fp64")
    base.update(kw)
    return ws.make_params(**base)


def test_plane_bytes_match_paper_table3():
    """FP64 path: 16-byte cells, so the Medium mesh is Table 3's 4.0 GB."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN,
                                                   "paper_table3_mesh.txt"))
            if ln.strip() and not ln.startswith("#")]
    medium = [r for r in rows if r[0] == "medium"][0]
    nu, nv, nw, gb = int(medium[1]), int(medium[2]), int(medium[3]), float(medium[4])
    pb, wb = ws.workspace_bytes(_p(nu=nu, nv=nv, nw=nw), 1 << 20)
    assert pb / 2 ** 30 == pytest.approx(gb, rel=1e-12)
    pb32, _ = ws.workspace_bytes(_p(nu=nu, nv=nv, nw=nw, precision="fp32"),
                                 1 << 20)
    assert pb32 * 2 == pb


def test_workspace_grows_with_max_vis():
    _, w1 = ws.workspace_bytes(_p(), 1000)
    _, w2 = ws.workspace_bytes(_p(), 100000)
    assert w2 > w1
    # records: at least key/rank (8) + cell (4) + 2 complex (32) + index (4)
    assert w2 - w1 >= 99000 * 48


@pytest.mark.parametrize("kw,status", [
    (dict(nu=500), _abi.WS_UNSUPPORTED_SIZE),
    (dict(nv=8), _abi.WS_UNSUPPORTED_SIZE),
    (dict(nu=65536), _abi.WS_UNSUPPORTED_SIZE),
    (dict(nv=65536), _abi.WS_UNSUPPORTED_SIZE),
    (dict(nw=0), _abi.WS_INVALID_ARG),
    (dict(support=6), _abi.WS_UNSUPPORTED_SIZE),
    (dict(support=17), _abi.WS_UNSUPPORTED_SIZE),
    (dict(fov_l=0.0), _abi.WS_INVALID_ARG),
    (dict(fov_l=float("nan")), _abi.WS_INVALID_ARG),
    (dict(fov_l=2.0, fov_m=2.0), _abi.WS_INVALID_ARG),
    (dict(w_min=1.0, w_max=1.0), _abi.WS_INVALID_ARG),
    (dict(w_max=float("inf")), _abi.WS_INVALID_ARG),
    (dict(precision=1, tile=48), _abi.WS_UNSUPPORTED_SIZE),
    (dict(tile=8), _abi.WS_UNSUPPORTED_SIZE),
    (dict(nu=16, nv=16, tile=16, support=17), _abi.WS_UNSUPPORTED_SIZE),
])
def test_invalid_params_rejected(kw, status):
    with pytest.raises(ws.WStackError) as ei:
        ws.validate(_p(**kw))
    assert ei.value.status == status
    assert len(str(ei.value)) > 20


def test_valid_edge_params_accepted():
    ws.validate(_p(nw=1, w_min=5.0, w_max=5.0))
    ws.validate(_p(nu=16, nv=16, support=15))
    ws.validate(_p(nu=4096, nv=16, support=1, tile=16))
    ws.validate(_p(nu=16384, nv=16384, precision="fp32"))
    ws.validate(_p(nu=16384, nv=16384, precision="fp64"))
    ws.validate(_p(nu=32768, nv=32768, precision="fp32"))
    ws.validate(_p(nu=32768, nv=32768, precision="fp64"))


def test_widest_rows_reserve_split_scratch():
    """FP64 rows of 32768 exceed two half-length LDS transforms: their
    plans reserve the 4-way split's scratch rows (256 rows of the grid
    width); FP32 rows of the same width do not need them."""
    _, w64 = ws.workspace_bytes(_p(nu=32768, nv=16, nw=1, precision="fp64",
                                   tile=16), 1000)
    _, w64n = ws.workspace_bytes(_p(nu=16384, nv=16, nw=1, precision="fp64",
                                    tile=16), 1000)
    assert w64 - w64n >= 256 * 32768 * 16
    _, w32 = ws.workspace_bytes(_p(nu=32768, nv=16, nw=1, precision="fp32",
                                   tile=16), 1000)
    assert w32 < 256 * 32768 * 8


def test_max_vis_bounds():
    with pytest.raises(ws.WStackError) as ei:
        ws.workspace_bytes(_p(), 0)
    assert ei.value.status == _abi.WS_INVALID_ARG
    with pytest.raises(ws.WStackError):
        ws.workspace_bytes(_p(), 1 << 31)


def test_null_and_status_strings():
    lib = ws.lib()
    assert lib.ws_validate_params(None) == _abi.WS_INVALID_ARG
    assert lib.ws_status_string(0) == b"WS_OK"
    assert lib.ws_status_string(_abi.WS_BAD_STATE) == b"WS_BAD_STATE"
    out = C.c_void_p(123)
    st = lib.ws_grid_init(C.byref(_p()), 10, None, 0, None, 0, None,
                          C.byref(out))
    assert st == _abi.WS_INVALID_ARG and out.value is None
    assert lib.ws_plan_reset(None) == _abi.WS_INVALID_ARG
    lib.ws_plan_destroy(None)


def test_noalloc_refuses_before_touching_a_device():
    """A problem larger than the static scratch is refused by the size
    check alone (no GPU here)."""
    p = _p(nu=4096, nv=4096, nw=32, precision="fp32")
    st = _abi.lib().ws_grid_image_noalloc(C.byref(p), 10, None, None, None,
                                          None, None, None)
    assert st == _abi.WS_WORKSPACE_TOO_SMALL
    msg = _abi.lib().ws_last_error().decode()
    assert "static scratch" in msg and str(64 << 20) in msg
    # and a bad parameter set is still reported as such
    bad = _p(nu=100)
    assert _abi.lib().ws_grid_image_noalloc(C.byref(bad), 10, None, None,
                                            None, None, None, None) == \
        _abi.WS_UNSUPPORTED_SIZE


# ---- production kernel and grid correction (host-only parts) -------------

@pytest.mark.parametrize("kernel", ["gauss", "es"])
@pytest.mark.parametrize("support", [1, 3, 7, 9, 15])
def test_kernel_transform_matches_oracle(kernel, support):
    """The library's psi (tanh-sinh quadrature) and kernel norm c against
    the oracle's (Gauss-Legendre after its own substitution), two
    independent quadratures of the same integral."""
    import numpy as np
    from oracle import wstack as o
    p = _p(support=support, kernel=kernel)
    po = o.Params(512, 512, 8, math.radians(1), math.radians(1), -100.0,
                  100.0, support, kernel=kernel)
    f = np.linspace(0.0, 0.5, 41)
    psi, c = ws.api.kernel_transform(p, f)
    ref = o.kernel_ft(po, f)
    # Relative to psi(0): where psi is small, both quadratures lose digits
    # to the cancellation of the oscillating integrand.
    assert np.abs(psi - ref).max() <= 1e-13 * ref[0]
    assert c == pytest.approx(o.kernel_norm(po), rel=1e-13)


def test_kernel_params_validated():
    ws.validate(_p(kernel="es", beta=0.0, correct=True))
    ws.validate(_p(kernel="es", beta=12.5))
    for bad in (dict(kernel=2), dict(beta=float("nan")), dict(beta=1e9),
                dict(correct=2)):
        p = _p()
        for k, v in bad.items():
            setattr(p, k, v)
        with pytest.raises(ws.WStackError) as e:
            ws.validate(p)
        assert e.value.status == _abi.WS_INVALID_ARG
    # A broad truncated Gaussian has a transform that changes sign inside
    # |f| <= 1/2: its correction is refused.
    with pytest.raises(ws.WStackError) as e:
        ws.validate(_p(support=7, sigma=6.0, correct=True))
    assert e.value.status == _abi.WS_INVALID_ARG
    ws.validate(_p(support=7, sigma=6.0, correct=False))
