"""C-ABI checks that need no GPU: the library loads, exports every function
include/pwa.h declares, and rejects bad arguments on the host with the
documented status codes before any HIP call is made.  No call here reaches
a kernel launch (fake device pointers only ever hit early validation)."""

import ctypes
import os
import re

import pytest

from paper_2403_09225_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(pwa_\w+)\s*\(", text))
    return sorted(names)


def _model(K=2, channel=None, spin=None):
    m = L.PwaModel()
    m.parent_mass = 1.865
    m.masses[0], m.masses[1], m.masses[2] = 0.494, 0.140, 0.140
    m.r = 3.0
    m.n_res = K
    m.width_mode = 0
    for k in range(K):
        m.channel[k] = (channel or [k % 3] * K)[k] if channel else k % 3
        m.spin[k] = spin[k] if spin else (k // 3) % 3
    return m


def _create(lib, m, streams=L.PWA_STREAM_F64):
    h = ctypes.c_void_p()
    code = lib.pwa_create(ctypes.byref(m), streams, ctypes.byref(h))
    return code, h


def test_every_declared_function_is_exported(lib):
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, n


def test_create_validation(lib):
    assert lib.pwa_create(None, 1, None) == L.PWA_E_INVALID
    for mutate in [
        lambda m: setattr(m, "n_res", 0),
        lambda m: setattr(m, "n_res", 65),
        lambda m: m.channel.__setitem__(0, 3),
        lambda m: m.spin.__setitem__(1, -1),
        lambda m: m.masses.__setitem__(0, 0.0),
        lambda m: setattr(m, "r", -1.0),
        lambda m: setattr(m, "parent_mass", 0.7),
        lambda m: setattr(m, "width_mode", 5),
        lambda m: setattr(m, "parent_mass", float("nan")),
    ]:
        m = _model()
        mutate(m)
        code, h = _create(lib, m)
        assert code == L.PWA_E_INVALID and not h.value
    code, h = _create(lib, _model(), streams=0)
    assert code == L.PWA_E_INVALID


def test_valid_context_host_queries(lib):
    code, h = _create(lib, _model(12), L.PWA_STREAM_F64 | L.PWA_STREAM_F32)
    assert code == L.PWA_OK
    try:
        assert lib.pwa_n_par(h) == 48
        assert lib.pwa_stream_fields(h) == 18   # 3 s, 6 u, 9 g planes
        assert lib.pwa_stream_fields(None) == -1
        assert lib.pwa_workspace_bytes(h, -1, 10) == 0
        assert lib.pwa_workspace_bytes(h, 10, 0) == 0
        a = lib.pwa_workspace_bytes(h, 1000, 5000)
        b = lib.pwa_workspace_bytes(h, 2000, 5000)
        # 18 planes (3 s, 6 u, 9 g) x (8 + 4) bytes per event for both streams
        assert b - a == pytest.approx(1000 * 18 * 12, abs=2 * 64 * 18 * 12 + 512)
        assert lib.pwa_grid_blocks(h) == -1
        assert lib.pwa_set_precision(h, L.PWA_PREC_F32) == L.PWA_OK
        assert lib.pwa_set_precision(h, 7) == L.PWA_E_INVALID
        assert lib.pwa_set_launch_shape(h, 1, 3, 3) == L.PWA_E_INVALID
        assert lib.pwa_set_launch_shape(h, 1, 1, 2) == L.PWA_E_INVALID   # 2 < K = 12
        assert lib.pwa_set_launch_shape(h, 3, 4, 3) == L.PWA_E_INVALID   # no layout 3
        assert lib.pwa_set_launch_shape(h, 1, 4, 3) == L.PWA_OK
        assert lib.pwa_set_launch_shape(h, 2, 4, 3) == L.PWA_OK
        assert lib.pwa_set_launch_shape(h, 2, 7, 3) == L.PWA_E_INVALID   # not built
        assert lib.pwa_set_launch_shape(h, 2, 8, 8) == L.PWA_OK
        assert lib.pwa_set_launch_shape(h, 0, 0, 0) == L.PWA_OK
    finally:
        lib.pwa_destroy(h)
    lib.pwa_destroy(None)


def test_f64_only_context_rejects_f32(lib):
    code, h = _create(lib, _model(2), L.PWA_STREAM_F64)
    assert code == L.PWA_OK
    assert lib.pwa_set_precision(h, L.PWA_PREC_F32) == L.PWA_E_INVALID
    lib.pwa_destroy(h)


def test_unbound_and_bad_bind_arguments(lib):
    code, h = _create(lib, _model(2))
    assert code == L.PWA_OK
    fake = ctypes.c_void_p(0x100000)
    st = None
    try:
        assert lib.pwa_nll(h, fake, fake, st) == L.PWA_E_STATE
        assert lib.pwa_grad(h, fake, fake, fake, st) == L.PWA_E_STATE
        assert lib.pwa_hvp(h, fake, fake, fake, None, None, st) == L.PWA_E_STATE
        assert lib.pwa_partials(h, fake, None, fake, st) == L.PWA_E_STATE
        assert lib.pwa_intensity(h, fake, 0, fake, st) == L.PWA_E_STATE
        assert lib.pwa_hessian(h, fake, fake, st) == L.PWA_E_STATE
        assert lib.pwa_hvp_reuse(h, fake, fake, None, None, st) == L.PWA_E_STATE
        nb = lib.pwa_fraction_matrix_workspace_bytes(h)
        assert nb > 0
        assert lib.pwa_fraction_matrix(h, fake, fake, nb, fake, st) == L.PWA_E_STATE
        assert lib.pwa_fraction_matrix(h, None, fake, nb, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_hvp_reuse(h, None, fake, None, None, st) == L.PWA_E_INVALID
        assert lib.pwa_partials_reuse(h, fake, fake, st) == L.PWA_E_STATE
        assert lib.pwa_partials_reuse(h, fake, None, st) == L.PWA_E_INVALID
        assert lib.pwa_hessian(h, None, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_fit_fractions(h, fake, fake, None, st) == L.PWA_E_STATE
        assert lib.pwa_fit_fractions(h, fake, None, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_intensity(h, fake, 2, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_intensity(h, None, 0, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_device_status(h, st) == L.PWA_E_STATE
        assert lib.pwa_nll(None, fake, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_nll(h, None, fake, st) == L.PWA_E_INVALID
        assert lib.pwa_hvp(h, fake, None, fake, None, None, st) == L.PWA_E_INVALID
        opts = L.PwaFitOpts()
        opts.xtol = 1e-8
        assert lib.pwa_fit(h, fake, ctypes.byref(opts), None, st) == L.PWA_E_STATE
        opts.reconjugate = 2
        assert lib.pwa_fit(h, fake, ctypes.byref(opts), None, st) in (L.PWA_E_STATE, L.PWA_E_INVALID)
        opts.reconjugate = 0
        assert lib.pwa_fit(h, fake, None, None, st) == L.PWA_E_INVALID
        assert lib.pwa_fit_bfgs(h, fake, ctypes.byref(opts), None, st) == L.PWA_E_STATE
        assert lib.pwa_fit_bfgs(h, fake, None, None, st) == L.PWA_E_INVALID
        assert lib.pwa_fit_bfgs(None, fake, ctypes.byref(opts), None, st) == L.PWA_E_INVALID
        need = lib.pwa_workspace_bytes(h, 10, 10)
        # n_mc < 1, negative n_data, null MC pointers
        assert lib.pwa_bind(h, fake, fake, 10, fake, fake, 0, fake, need, st) == L.PWA_E_INVALID
        assert lib.pwa_bind(h, fake, fake, -1, fake, fake, 10, fake, need, st) == L.PWA_E_INVALID
        assert lib.pwa_bind(h, fake, fake, 10, None, fake, 10, fake, need, st) == L.PWA_E_INVALID
        assert lib.pwa_bind(h, None, fake, 10, fake, fake, 10, fake, need, st) == L.PWA_E_INVALID
        # workspace: null, misaligned, too small
        assert lib.pwa_bind(h, fake, fake, 10, fake, fake, 10, None, need, st) == L.PWA_E_WORKSPACE
        assert lib.pwa_bind(h, fake, fake, 10, fake, fake, 10, ctypes.c_void_p(0x100001), need,
                            st) == L.PWA_E_WORKSPACE
        assert lib.pwa_bind(h, fake, fake, 10, fake, fake, 10, fake, need - 1, st) == L.PWA_E_WORKSPACE
    finally:
        lib.pwa_destroy(h)


def test_combine_validation(lib):
    fake = ctypes.c_void_p(0x100000)
    assert lib.pwa_combine(5, 1, fake, 10, 10, None, fake, None, None, None) == L.PWA_E_INVALID
    assert lib.pwa_combine(8, 0, fake, 10, 10, None, fake, None, None, None) == L.PWA_E_INVALID
    assert lib.pwa_combine(8, 1, None, 10, 10, None, fake, None, None, None) == L.PWA_E_INVALID
    assert lib.pwa_combine(8, 1, fake, 10, 0, None, fake, None, None, None) == L.PWA_E_INVALID
    assert lib.pwa_combine(8, 1, fake, 10, 10, None, fake, fake, fake, None) == L.PWA_E_INVALID


def test_status_strings(lib):
    for code in range(-6, 1):
        s = lib.pwa_status_str(code)
        assert s and len(s) >= 2
    assert b"unknown" in lib.pwa_status_str(-99)


def test_mlp_host_validation(lib):
    d = L.PwaMlpDims(1024, 512, 512, 48)
    assert lib.pwa_mlp_n_params(ctypes.byref(d)) == 512 * 1024 + 512 + 512 * 512 + 512 + 48 * 512 + 48
    assert lib.pwa_mlp_n_transposed(ctypes.byref(d)) == 512 * 512 + 512 * 48
    bad = L.PwaMlpDims(1000, 512, 512, 48)
    assert lib.pwa_mlp_n_params(ctypes.byref(bad)) == 0
    assert lib.pwa_mlp_workspace_bytes(ctypes.byref(bad), 16) == 0
    nb = lib.pwa_mlp_workspace_bytes(ctypes.byref(d), 100)
    assert nb > 0 and nb == lib.pwa_mlp_workspace_bytes(ctypes.byref(d), 112)
    fake = ctypes.c_void_p(0x1000)
    st = None
    assert lib.pwa_mlp_forward(ctypes.byref(d), fake, fake, None, 4, fake, fake, nb, st) == L.PWA_E_INVALID
    assert lib.pwa_mlp_forward(ctypes.byref(d), fake, fake, fake, 0, fake, fake, nb, st) == L.PWA_E_INVALID
    assert lib.pwa_mlp_forward(ctypes.byref(d), fake, fake, fake, 4, fake, fake, 16, st) == L.PWA_E_WORKSPACE
    assert lib.pwa_mlp_backward(ctypes.byref(bad), fake, fake, fake, 4, fake, nb, fake, fake, st) == L.PWA_E_INVALID
    assert lib.pwa_mlp_adam(ctypes.byref(d), fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8,
                            0.0, fake, fake, st) == L.PWA_E_INVALID
    assert lib.pwa_mlp_adam(ctypes.byref(d), fake, fake, fake, fake, 1, 1e-3, 0.9, 0.999, 1e-8,
                            -1.0, fake, fake, st) == L.PWA_E_INVALID
    masses = (ctypes.c_double * 3)(0.494, 0.140, 0.140)
    assert lib.pwa_hist2d(fake, fake, fake, 0, 1.865, masses, fake, st) == L.PWA_E_INVALID
    assert lib.pwa_hist2d(fake, fake, fake, 1, 0.5, masses, fake, st) == L.PWA_E_INVALID


def test_event_count_limit(lib):
    """Planes are addressed with 32-bit byte offsets: at most 2^29 - 256
    events per context (FP64 stream); beyond that the workspace query returns
    0 and bind rejects the sizes before any device call."""
    code, h = _create(lib, _model())
    assert code == L.PWA_OK
    try:
        lim = (1 << 29) - 256
        assert lib.pwa_workspace_bytes(h, lim - 10, 10) > 0
        assert lib.pwa_workspace_bytes(h, lim - 9, 10) == 0
        fake = ctypes.c_void_p(0x1000)
        assert lib.pwa_bind(h, fake, fake, lim, fake, fake, 10, fake, 1 << 40, None) == L.PWA_E_INVALID
    finally:
        lib.pwa_destroy(h)


# ------------------------------------------------ host-only error matrix
def _spd(P, seed):
    import numpy as np
    r = np.random.Generator(np.random.PCG64(seed))
    A = r.normal(size=(P, P))
    return A @ A.T + P * np.eye(P)


def test_covariance_is_inverse_of_free_block():
    """pwa_covariance (Cholesky on the host) against numpy's inverse of the
    free block; fixed rows and columns are zero and the result is exactly
    symmetric."""
    import numpy as np
    from paper_2403_09225_amd.api import covariance
    for P, seed in ((4, 1), (12, 2), (48, 3), (120, 4)):
        H = _spd(P, seed)
        free = np.random.Generator(np.random.PCG64(seed + 10)).random(P) > 0.2
        C = covariance(H, free)
        ref = np.zeros((P, P))
        ref[np.ix_(free, free)] = np.linalg.inv(H[np.ix_(free, free)])
        np.testing.assert_allclose(C, ref, rtol=1e-10, atol=1e-13 * np.max(np.abs(ref)))
        assert np.array_equal(C, C.T)
        np.testing.assert_allclose(covariance(H), np.linalg.inv(H), rtol=1e-10,
                                   atol=1e-13 * np.max(np.abs(np.linalg.inv(H))))


def test_covariance_errors(lib):
    import numpy as np
    from paper_2403_09225_amd.api import covariance
    H = _spd(8, 5)
    H[3, 3] = -1.0                       # not positive definite
    with pytest.raises(L.PwaError):
        covariance(H)
    fm = np.ones(8, bool)
    fm[3] = False
    covariance(H, fm)                    # fine once that parameter is fixed
    Hn = _spd(8, 6)
    Hn[1, 2] = np.nan
    out = np.empty((8, 8))
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.pwa_covariance(8, ptr(Hn), None, ptr(out)) == L.PWA_E_INVALID
    assert lib.pwa_covariance(0, ptr(Hn), None, ptr(out)) == L.PWA_E_INVALID
    assert lib.pwa_covariance(8, None, None, ptr(out)) == L.PWA_E_INVALID
    # the likelihood's symmetry makes the all-free Hessian singular; with a
    # zero mode pushed slightly negative by rounding, Cholesky must refuse
    A = np.random.Generator(np.random.PCG64(7)).normal(size=(8, 7))
    u = np.linalg.svd(A.T)[2][-1]            # null vector of A^T
    Z = np.ascontiguousarray(A @ A.T - 1e-9 * np.outer(u, u))
    assert lib.pwa_covariance(8, ptr(Z), None, ptr(out)) == L.PWA_E_DOMAIN
    # ... and also when rounding pushes it slightly positive: a pivot within
    # the rounding of the elimination is a zero direction, not a tiny variance
    for eps in (1e-15, 1e-14):
        Zp = np.ascontiguousarray(A @ A.T + eps * np.outer(u, u))
        assert lib.pwa_covariance(8, ptr(Zp), None, ptr(out)) == L.PWA_E_DOMAIN
    # a genuinely ill-conditioned but positive definite block is still inverted
    Zc = np.ascontiguousarray(A @ A.T + 1e-6 * np.outer(u, u))
    assert lib.pwa_covariance(8, ptr(Zc), None, ptr(out)) == L.PWA_OK
    np.testing.assert_allclose(out, np.linalg.inv(Zc), rtol=1e-6, atol=1e-6 * np.abs(out).max())


def test_propagate():
    import numpy as np
    from paper_2403_09225_amd.api import propagate
    C = np.linalg.inv(_spd(10, 8))
    J = np.random.Generator(np.random.PCG64(9)).normal(size=(4, 10))
    np.testing.assert_allclose(propagate(J, C), np.sqrt(np.einsum("ri,ij,rj->r", J, C, J)),
                               rtol=1e-13)
    assert propagate(np.zeros((1, 10)), C)[0] == 0.0


def test_fraction_matrix_limits(lib):
    """The Gram route serves K <= 24 with an FP64 event stream only."""
    for K, streams, ok in ((24, L.PWA_STREAM_F64, True), (25, L.PWA_STREAM_F64, False),
                           (6, L.PWA_STREAM_F32, False)):
        code, h = _create(lib, _model(K), streams)
        assert code == L.PWA_OK
        try:
            assert (lib.pwa_fraction_matrix_workspace_bytes(h) > 0) == ok
        finally:
            lib.pwa_destroy(h)


def test_general_physics_model_validation(lib):
    """Flatte only for scalars, its second channel and ratio valid, a parent
    spin of 0 or 1, at most 16 resonances on the general path; each bind
    entry point serves its own parent spin and layout 3 its own models.
    All rejected on the host, before any device call."""
    fake = ctypes.c_void_p(0x1000)
    m = _model(2, spin=[0, 1])
    m.lineshape[1] = L.PWA_LINESHAPE_FLATTE          # J = 1: not a scalar
    m.flatte_masses[0] = m.flatte_masses[1] = 0.4937
    m.flatte_ratio = 4.0
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m = _model(2, spin=[0, 1])
    m.lineshape[0] = L.PWA_LINESHAPE_FLATTE
    m.flatte_ratio = 4.0                              # second-channel masses unset
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m.flatte_masses[0] = m.flatte_masses[1] = 0.4937
    m.flatte_ratio = -1.0
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m.flatte_ratio = 4.0
    m.lineshape[1] = 7
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m.lineshape[1] = 0
    code, h = _create(lib, m)
    assert code == L.PWA_OK
    try:
        assert lib.pwa_set_launch_shape(h, 2, 1, 2) == L.PWA_E_INVALID
        assert lib.pwa_set_launch_shape(h, 3, 1, 2) == L.PWA_OK
        assert lib.pwa_set_launch_shape(h, 3, 3, 2) == L.PWA_E_INVALID   # not built
        assert lib.pwa_set_launch_shape(h, 3, 4, 3) == L.PWA_OK
        assert lib.pwa_set_launch_shape(h, 3, 8, 3) == L.PWA_E_INVALID   # not built
        assert lib.pwa_bind_oriented(h, fake, fake, fake, fake, 10, fake, fake, fake, fake, 10,
                                     fake, 1 << 30, None) == L.PWA_E_INVALID
    finally:
        lib.pwa_destroy(h)
    m = _model(3)
    m.parent_spin = 2
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m.parent_spin = 1
    code, h = _create(lib, m)
    assert code == L.PWA_OK
    try:
        assert lib.pwa_bind(h, fake, fake, 10, fake, fake, 10, fake, 1 << 30, None) == L.PWA_E_INVALID
        # orientation arrays are required
        assert lib.pwa_bind_oriented(h, fake, fake, None, fake, 10, fake, fake, fake, fake, 10,
                                     fake, 1 << 30, None) == L.PWA_E_INVALID
        assert lib.pwa_fraction_matrix_workspace_bytes(h) == 0
    finally:
        lib.pwa_destroy(h)
    m = _model(17)
    m.parent_spin = 1
    assert _create(lib, m)[0] == L.PWA_E_INVALID
    m = _model(17)
    code, h = _create(lib, m)
    assert code == L.PWA_OK
    lib.pwa_destroy(h)
