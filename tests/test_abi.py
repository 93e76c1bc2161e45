"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects invalid arguments on the host before any
HIP call (so fake, never-dereferenced device pointers are safe here)."""
import ctypes
import json
import math
import os
import re

import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcasolve.h")

FAKE = ctypes.c_void_p(0x100000)       # aligned, never dereferenced
EINVAL, EGEOM, ESING, ENONFIN, EWS = -1, -2, -3, -4, -5


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_1102_1712_amd import build
        build.build()
    return B.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path_entry_points():
    names = _declared_functions()
    for n in ("pca_dvf", "warp_trilinear", "drr_forward", "drr_adjoint", "grad_w",
              "solve_projection", "ray_table", "residual_fit", "tumour_position"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), f"{n} declared in pcasolve.h but not exported"
    assert set(B.EXPORTS) <= set(names)


def test_abi_version_and_status_strings(L):
    assert L.pcas_abi_version() == 8
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.pcas_status_string(code)
    assert L.pcas_last_error() == b""


def test_kernel_classes_match_the_header():
    """The binding's kernel-class names and profile mask follow the header's
    PCAS_K_* enumeration."""
    src = open(os.path.join(ROOT, "include", "pcasolve.h")).read()
    ids = {m.group(1): int(m.group(2)) for m in re.finditer(r"PCAS_K_(\w+) = (\d+)", src)}
    n = ids.pop("CLASSES")
    assert n == len(B.KERNEL_CLASSES) and sorted(ids.values()) == list(range(n))
    assert "#define PCAS_PROFILE_ALL ((1 << PCAS_K_CLASSES) - 1)" in src
    assert B.PROFILE_ALL == (1 << n) - 1 == B.profile_mask()
    assert B.profile_mask("drr_adjoint_chain") == 1 << ids["ADJOINT"]
    assert B.profile_mask("spec_skipped", "warp_pca") == (1 << ids["SPEC_SKIP"]) | (1 << ids["WARP"])


def test_default_and_paper_options(L):
    o = B.default_opts()
    assert (o.method, o.max_iter, o.fit_intensity, o.max_backtracks) == (1, 30, 1, 12)
    assert (o.mu0, o.alpha, o.beta, o.beta_lo) == (1.0, 0.1, 0.5, 0.1)
    assert o.grad_mode == 1 and o.ls_extrap == 10.0 and o.ftol_rel < 0
    assert o.polish == 1 and o.speculate == 1
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    p = B.paper_opts()
    scale = 1.0 / g["coefficient_std"]
    assert p.method == 0 and p.max_iter == g["max_iter"]
    assert p.alpha == g["armijo_alpha"] and p.beta == g["armijo_beta"]
    assert math.isclose(p.mu0, g["armijo_mu0"] * scale) and math.isclose(p.mu_min, g["stop_step"] * scale)


def _vp(case):
    return B.c_vol(case.vol), B.c_proj(case.proj)


@pytest.fixture(scope="module")
def geom():
    vol = synth.centred_volume((20, 18, 16), (4.0, 4.0, 5.0))
    proj = synth.Projection(angle=0.3, sad=1000.0, sid=1500.0, nu=32, nv=24, pitch_u=3.0,
                            pitch_v=3.0, step=2.0)
    return B.c_vol(vol), B.c_proj(proj)


def test_ray_table_bytes(L, geom):
    v, p = geom
    assert L.pcas_ray_table_bytes(0, ctypes.byref(p)) == 32 * 32 * 24
    assert L.pcas_ray_table_bytes(1, ctypes.byref(p)) == 64 * 32 * 24
    assert L.pcas_ray_table_bytes(7, ctypes.byref(p)) == 0


def test_backprojection_brick_count(L, geom):
    """Bricks tile the volume 32 x 16 x 8 (x, y, z), ragged edges rounded up."""
    v, _ = geom
    assert L.backprojection_brick_count(ctypes.byref(v)) == 1 * 2 * 2
    odd = B.c_vol(synth.centred_volume((65, 17, 9), (1.0, 1.0, 1.0)))
    assert L.backprojection_brick_count(ctypes.byref(odd)) == 3 * 2 * 2
    assert B.backprojection_brick_count(synth.centred_volume((256, 256, 128), (1.0, 1.0, 1.0))) == 8 * 16 * 16


def test_invalid_dtype_dims_and_pointers(L, geom):
    v, p = geom
    assert L.ray_table(7, ctypes.byref(v), ctypes.byref(p), FAKE, None) == EINVAL
    bad = B.Vol()
    ctypes.memmove(ctypes.byref(bad), ctypes.byref(v), ctypes.sizeof(v))
    bad.n[1] = 1
    assert L.ray_table(0, ctypes.byref(bad), ctypes.byref(p), FAKE, None) == EINVAL
    bad.n[1] = 18
    bad.spacing[2] = 0.0
    assert L.drr_forward(0, ctypes.byref(bad), ctypes.byref(p), FAKE, FAKE, FAKE, None) == EINVAL
    assert L.ray_table(0, ctypes.byref(v), ctypes.byref(p), None, None) == EINVAL
    assert L.ray_table(0, ctypes.byref(v), ctypes.byref(p), ctypes.c_void_p(0x100004), None) == EINVAL
    assert L.drr_adjoint(0, ctypes.byref(v), ctypes.byref(p), FAKE, None, FAKE, None) == EINVAL
    w = (ctypes.c_double * 3)(0.1, 0.2, 0.3)
    assert L.pca_dvf(0, 100, 0, None, FAKE, w, FAKE, None) == EINVAL
    assert L.pca_dvf(0, 100, 9, None, FAKE, w, FAKE, None) == EINVAL
    assert L.warp_trilinear(0, ctypes.byref(v), FAKE, FAKE, FAKE, None) == EINVAL   # f_out aliases f0


def test_volume_over_2gib_rejected(L, geom):
    """Kernels address a volume with 32-bit byte offsets."""
    _, p = geom
    big = B.c_vol(synth.centred_volume((1024, 1024, 512), (0.5, 0.5, 0.5)))
    assert L.ray_table(0, ctypes.byref(big), ctypes.byref(p), FAKE, None) == EINVAL
    half = B.c_vol(synth.centred_volume((1024, 1024, 256), (0.5, 0.5, 0.5)))
    assert L.drr_forward(1, ctypes.byref(half), ctypes.byref(p), FAKE, FAKE, FAKE, None) == EINVAL


def test_invalid_geometry(L, geom):
    v, p = geom
    for field, val in (("sad", 0.0), ("sid", 900.0), ("pitch_u", 0.0), ("step", -1.0),
                       ("angle", float("nan"))):
        q = B.Proj()
        ctypes.memmove(ctypes.byref(q), ctypes.byref(p), ctypes.sizeof(p))
        setattr(q, field, val)
        assert L.ray_table(0, ctypes.byref(v), ctypes.byref(q), FAKE, None) == EGEOM, field
    # a source orbit that passes through the volume
    q = B.Proj()
    ctypes.memmove(ctypes.byref(q), ctypes.byref(p), ctypes.sizeof(p))
    q.sad, q.sid = 30.0, 60.0
    assert L.drr_forward(0, ctypes.byref(v), ctypes.byref(q), FAKE, FAKE, FAKE, None) == EGEOM


def test_nonfinite_coefficients_rejected(L, geom):
    v, _ = geom
    w = (ctypes.c_double * 3)(0.1, float("nan"), 0.3)
    assert L.warp_pca(0, ctypes.byref(v), 3, FAKE, None, FAKE, w, ctypes.c_void_p(0x200000), None) == ENONFIN
    assert L.pca_dvf(1, 100, 3, None, FAKE, w, FAKE, None) == ENONFIN
    c0 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert L.tumour_position(0, ctypes.byref(v), 3, None, FAKE, w, c0, 1e-9, 100, FAKE, None) == ENONFIN


def test_workspace_checks(L, geom):
    v, p = geom
    need = L.grad_w_workspace_bytes(0, ctypes.byref(v), 3)
    assert need > 0
    w = (ctypes.c_double * 3)(0.1, 0.2, 0.3)
    assert L.grad_w(0, ctypes.byref(v), 3, FAKE, None, FAKE, w, FAKE, FAKE, FAKE, need - 1, None) == EWS
    assert L.grad_w(0, ctypes.byref(v), 3, FAKE, None, FAKE, w, FAKE, FAKE, None, need, None) == EWS
    assert L.residual_fit(0, 1000, FAKE, FAKE, 1, None, FAKE, FAKE, 16, None) == EWS
    ws = L.solve_projection_workspace(0, ctypes.byref(v), ctypes.byref(p), 3)
    # rays (32 B/pixel) + f, bp (4 B/voxel) + p (4 B/pixel) + reduction scratch
    assert ws >= 32 * 768 + 2 * 4 * 5760 + 4 * 768
    o = B.default_opts()
    rep = B.Report()
    wout = (ctypes.c_double * 3)()
    args = [0, ctypes.byref(v), ctypes.byref(p), 3, FAKE, None, FAKE, FAKE, w, ctypes.byref(o)]
    assert L.solve_projection(*args, FAKE, ws - 256, wout, ctypes.byref(rep), None) == EWS
    assert L.solve_projection(*args, ctypes.c_void_p(0x100010), ws, wout, ctypes.byref(rep), None) == EWS


def test_solve_option_and_input_validation(L, geom):
    v, p = geom
    ws = L.solve_projection_workspace(1, ctypes.byref(v), ctypes.byref(p), 3)
    rep = B.Report()
    wout = (ctypes.c_double * 3)()
    good_w = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    nan_w = (ctypes.c_double * 3)(0.0, float("inf"), 0.0)

    def call(o, w=good_w, K=3):
        return L.solve_projection(1, ctypes.byref(v), ctypes.byref(p), K, FAKE, None, FAKE, FAKE, w,
                                  ctypes.byref(o), FAKE, ws, wout, ctypes.byref(rep), None)

    assert call(B.default_opts(), w=nan_w) == ENONFIN
    assert call(B.default_opts(method=3)) == EINVAL
    assert call(B.default_opts(method=-1)) == EINVAL
    assert call(B.default_opts(ls_extrap=-1.0)) == EINVAL
    assert call(B.default_opts(ls_extrap=float("inf"))) == EINVAL
    assert call(B.default_opts(ftol_rel=float("nan"))) == EINVAL
    assert call(B.default_opts(alpha=1.5)) == EINVAL
    assert call(B.default_opts(beta=0.0)) == EINVAL
    assert call(B.default_opts(mu0=0.0)) == EINVAL
    assert call(B.default_opts(max_backtracks=0)) == EINVAL
    assert call(B.default_opts(beta_lo=0.9)) == EINVAL
    assert call(B.default_opts(locate=1, c0_mm=(0.0, float("nan"), 0.0))) == EINVAL
    assert call(B.default_opts(), K=0) == EINVAL
    assert call(B.default_opts(grad_mode=3)) == EINVAL
    assert call(B.default_opts(profile=-1)) == EINVAL
    assert call(B.default_opts(profile=B.PROFILE_ALL + 1)) == EINVAL
    assert L.solve_projection(1, ctypes.byref(v), ctypes.byref(p), 3, FAKE, None, FAKE, FAKE, good_w,
                              None, FAKE, ws, wout, ctypes.byref(rep), None) == EINVAL


def test_objective_gradient_validation(L, geom):
    v, p = geom
    ws = L.solve_projection_workspace(0, ctypes.byref(v), ctypes.byref(p), 3)
    # the workspace holds the K Jacobian volumes
    assert ws >= 3 * 4 * 5760 + 4 * 5760
    assert L.solve_projection_workspace(0, ctypes.byref(v), ctypes.byref(p), 0) == 0
    w = (ctypes.c_double * 3)(0.1, 0.2, 0.3)
    out = (ctypes.c_double * 6)()

    def call(K=3, w=w, mode=0, ws_ptr=FAKE, ws_bytes=ws):
        return L.objective_gradient(0, ctypes.byref(v), ctypes.byref(p), K, FAKE, None, FAKE, FAKE,
                                    w, 1, mode, ws_ptr, ws_bytes, out, None)

    assert call(mode=3) == EINVAL
    assert call(K=9) == EINVAL
    assert call(w=(ctypes.c_double * 3)(0.1, float("nan"), 0.3)) == ENONFIN
    assert call(ws_bytes=ws - 1) == EWS
    assert call(ws_ptr=ctypes.c_void_p(0x100010)) == EWS
    assert L.objective_gradient(0, ctypes.byref(v), ctypes.byref(p), 3, FAKE, None, FAKE, FAKE, w,
                                1, 0, FAKE, ws, None, None) == EINVAL


def test_server_validation(L):
    """Argument checks that return before any HIP call."""
    out = ctypes.c_void_p()
    assert L.pcas_server_create(None, 1 << 20, 4, None, ctypes.byref(out)) == EINVAL
    assert L.pcas_server_create(ctypes.c_void_p(0x100010), 1 << 20, 4, None,
                                ctypes.byref(out)) == EINVAL          # misaligned
    assert L.pcas_server_create(FAKE, 1 << 20, 0, None, ctypes.byref(out)) == EINVAL
    small = L.pcas_server_reserved_bytes(4)
    assert small > 0 and L.pcas_server_reserved_bytes(0) == 0
    assert L.pcas_server_create(FAKE, small, 4, None, ctypes.byref(out)) == EWS
    assert L.pcas_server_step(None, None) == EINVAL
    assert L.pcas_server_set_substep_share(None, 0.25) == EINVAL
    assert L.pcas_server_destroy(None) == EINVAL
    assert L.pcas_server_request_bytes(None, 0, None, None) == 0
