"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
entry point include/pyhst.h declares, and rejects invalid input before touching
the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1306_1392_amd as ph
from paper_1306_1392_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pyhst.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s*([A-Za-z_]\w*)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert {"fbp_filter", "backproject", "forward_project", "tv_prox", "reconstruct_slices"} <= set(names)
    L = ph.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_strerror():
    L = ph.lib()
    assert L.pyhst_strerror(0) == b"ok"
    assert L.pyhst_strerror(-2) == b"invalid geometry"


def _plan_rc(geo, n_slices=1, slice_geom=None):
    arr = (_lib.Geom * 1)(geo._c()) if isinstance(geo, ph.Geometry) else geo
    h = ctypes.c_void_p()
    rc = ph.lib().pyhst_plan_create(arr, 1, slice_geom, n_slices, ctypes.byref(h))
    return rc


def test_invalid_geometry_rejected_on_host():
    K = 90
    ang = ph.uniform_angles(K)
    assert _plan_rc(ph.Geometry(0, 8, 8, ang, 3.5)) == _lib.EARG
    assert _plan_rc(ph.Geometry(8, 8, 8, ang, 9.0)) == _lib.EARG              # axis outside the detector
    assert _plan_rc(ph.Geometry(8, 8, 8, ang[:45], 3.5)) == _lib.EGEOM        # 90 degrees only (section 2.1)
    assert _plan_rc(ph.Geometry(8, 8, 8, ang, 3.5, scan=ph.SCAN_360)) == _lib.EGEOM
    bad = ang.copy()
    bad[3] = np.nan
    assert _plan_rc(ph.Geometry(8, 8, 8, bad, 3.5)) == _lib.EARG
    # half acquisition: axis must be in the outer quarter of the detector
    ang2 = ph.uniform_angles(180, 2 * math.pi)
    assert _plan_rc(ph.Geometry(8, 8, 40, ang2, 20.0, scan=ph.SCAN_360_HALF)) == _lib.EGEOM
    assert _plan_rc(ph.Geometry(8, 8, 40, ang2, 35.0, scan=ph.SCAN_360_HALF, ha_overlap=6.0)) == _lib.EARG
    assert _plan_rc(ph.Geometry(8, 8, 8, ang, 3.5), n_slices=0) == _lib.EARG
    assert _plan_rc(ph.Geometry(46341, 46341, 8, ang, 3.5)) == _lib.EARG           # 2^31 pixels per slice
    assert b"2^31" in ph.lib().pyhst_last_error()
    assert _plan_rc(ph.Geometry(8, 8, 8, ang, 3.5), n_slices=65536) == _lib.EARG    # one grid dimension
    assert b"65535" in ph.lib().pyhst_last_error()
    assert b"cover" in ph.lib().pyhst_last_error() or b"slices" in ph.lib().pyhst_last_error()


def test_fake_oom_injection(monkeypatch):
    monkeypatch.setenv("PYHST_FAKE_OOM", "1")
    assert _plan_rc(ph.Geometry(8, 8, 8, ph.uniform_angles(90), 3.5)) == _lib.ENOMEM


def test_null_arguments():
    L = ph.lib()
    assert L.fbp_filter(None, None, None, None) == _lib.EARG
    assert L.backproject(None, None, 0, None, 1.0, 0.0, None) == _lib.EARG
    assert L.forward_project(None, None, None, 1.0, None) == _lib.EARG
    assert L.pyhst_opnorm(None, 1, 1.0, None, None, None, None) == _lib.EARG
    assert L.pyhst_plan_set_bp_slices(None, 2) == _lib.EARG
    assert L.pyhst_patch_fista(None, None, None) == _lib.EARG
    assert L.pyhst_patch_lipschitz(None, None, None) == _lib.EARG
    assert L.pyhst_unet_set_scale(None, 1.0) == _lib.EARG
    assert L.pyhst_cv_error(None, None, None, 0, None, None, 1.0, 0, None) == _lib.EARG
    assert L.tv_prox(1, 4, 4, None, None, 0.1, 10, None, 0, None) == _lib.EARG
    # too many slices: rejected on the host before any pointer is used
    assert L.tv_prox(65536, 4, 4, 16, 16, 0.1, 10, 16, 1 << 40, None) == _lib.EARG
    assert L.reconstruct_slices(None, None, None) == _lib.EARG


def test_product_path_has_no_oracle_import():
    """The reconstruction package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_1306_1392_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, f


class _FakePlan:
    """Stands in for a plan on the host: the wrappers validate buffers before any device call."""
    def __init__(self, R=2, K=6, nb=8, n=8):
        self.geom0 = ph.Geometry(n, n, nb, ph.uniform_angles(K), (nb - 1) / 2)
        self.n_slices = R
        self.sino_elems = R * K * nb
        self.img_elems = R * n * n
        self.filt_elems = self.sino_elems
        self.uniform = True

    def sino_shape(self):
        return (self.n_slices, self.geom0.n_angles, self.geom0.n_det)

    def img_shape(self):
        return (self.n_slices, self.geom0.n_y, self.geom0.n_x)


def test_raw_wrappers_validate_flats_and_dark():
    """Raw input: flats [n_flats][R][n_det] and dark [R][n_det] float32, contiguous, are checked before the
    library is called (the kernels index them by those sizes)."""
    import torch
    P = _FakePlan()
    R, K, nb = 2, 6, 8
    raw = torch.zeros((K, R, nb), dtype=torch.uint16)
    good_f, good_d, fp = torch.zeros((2, R, nb)), torch.zeros((R, nb)), [0.0, K - 1.0]
    bad = [(torch.zeros((2, R, nb - 1)), good_d, "flats"), (torch.zeros((1, R, nb)), good_d, "flats"),
           (good_f.double(), good_d, "flats"), (good_f, torch.zeros((R, nb + 1)), "dark"),
           (good_f, torch.zeros((nb, R)).t(), "dark"), (good_f, None, "dark")]
    for f, d, name in bad:
        for call in (lambda: ph.api.pyhst_normalize(P, raw, f, fp, d),
                     lambda: ph.api.normalize_hotspot(P, raw, f, fp, d, 0.1),
                     lambda: ph.reconstruct_slices(P, raw=raw, flats=f, flat_pos=fp, dark=d)):
            with pytest.raises((ValueError, TypeError), match=name):
                call()
    # halo rows: raw, flats and dark then hold R + 2 rows
    with pytest.raises(ValueError, match="raw"):
        ph.api.normalize_hotspot(P, raw, good_f, fp, good_d, 0.1, halo=(1, 1))
