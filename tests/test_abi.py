"""The C-ABI library loads and exports every entry point gd.h declares; its
argument checks run on the host (no GPU call is made here)."""

import ctypes
import os
import re

import pytest

import paper_1310_0041_amd as gd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return gd.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gd.exported_symbols())


def test_defaults(lib):
    o = gd.default_opts()
    # sweeps per cycle left to the library (-1: chosen per storage path at the call)
    assert o.rel_tol == 1e-6 and o.pre_smooth == -1 and o.post_smooth == -1 and o.storage == gd.F32
    assert lib.gd_version().startswith(b"gdstack")


P = ctypes.c_void_p


@pytest.mark.parametrize(
    "args,status",
    [
        ((None, 1, P(64), 1, 4, 4, 4, 1.0, 1.0, 4.0), gd.ERR_INVALID),          # null input
        ((P(64), 1, P(64), 1, 4, 4, 4, 1.0, 1.0, 4.0), gd.ERR_INVALID),         # aliasing
        ((P(64), 1, P(128), 1, 0, 4, 4, 1.0, 1.0, 4.0), gd.ERR_INVALID),        # empty
        ((P(64), 1, P(128), 1, 4, 4, 4, 1.0, 1.0, 0.0), gd.ERR_INVALID),        # beta_z = 0
        ((P(64), 1, P(128), 1, 4, 4, 4, -1.0, 1.0, 4.0), gd.ERR_INVALID),       # negative beta
        ((P(64), 1, P(128), 1, 4, 4, 4, float("nan"), 1.0, 4.0), gd.ERR_INVALID),
        ((P(64), 7, P(128), 1, 4, 4, 4, 1.0, 1.0, 4.0), gd.ERR_INVALID),        # bad dtype
        ((P(64), 1, P(128), 1, 4, 4, 2**31, 1.0, 1.0, 4.0), gd.ERR_INVALID),    # too long
    ],
)
def test_smooth_z_argument_checks(lib, args, status):
    assert lib.gd_smooth_z(*args, None, None, None) == status
    assert lib.gd_last_error()


def test_option_checks(lib):
    base = (P(64), 1, P(128), 1, 4, 4, 4, 1.0, 1.0, 4.0)
    for kw, st in [
        (dict(storage=gd.F16), gd.ERR_UNSUPPORTED),
        (dict(storage=gd.BF16), gd.ERR_UNSUPPORTED),
        (dict(rel_tol=0.0), gd.ERR_INVALID),
        (dict(pre_smooth=0, post_smooth=0), gd.ERR_INVALID),
        (dict(prolong=3), gd.ERR_INVALID),
        (dict(storage=9), gd.ERR_INVALID),
    ]:
        o = gd.default_opts(**kw)
        assert lib.gd_smooth_z(*base, ctypes.byref(o), None, None) == st, kw


def test_slice_argument_checks(lib):
    d = gd.make_slice_descs([0, 50], 10, 10, 0.01)
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 1, d, 2, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # slices overlap
    d = gd.make_slice_descs([0, 100], 10, 10, 0.0)
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 1, d, 2, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # alpha must be > 0
    d = gd.make_slice_descs([0], 10, 10, 0.01, pitch=[5])
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 1, d, 1, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # pitch < nx
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(64), 1, d, 1, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # aliasing
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 1, d, -1, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # negative count
    d = gd.make_slice_descs([0], 10, 10, 0.01)
    for t1 in (gd.F16, gd.BF16, 9):  # I1 must have I0's dtype, F32 or F64
        assert lib.gd_screened_poisson_slices(P(64), gd.F64, P(128), t1, P(256), 1, d, 1, 1.0, 1.0, None, None,
                                              None, None) == gd.ERR_INVALID
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 7, d, 1, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_INVALID  # bad output dtype
    rep = gd.Report()
    rep.cycles = 7
    assert lib.gd_screened_poisson_slices(None, 1, None, 1, None, 1, None, 0, 1.0, 1.0, None, ctypes.byref(rep),
                                          None, None) == gd.OK  # an empty batch touches nothing
    assert rep.cycles == 0


def test_npr_argument_checks(lib):
    def call(alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.25, sigma=5.0, opts=None, out=P(128)):
        return lib.gd_npr_filter(P(64), 1, out, 1, 8, 8, 4, alpha, beta[0], beta[1], beta[2], lam, sigma, opts,
                                 None, None)
    assert call(alpha=0.0) == gd.ERR_INVALID
    assert call(beta=(1.0, -1.0, 0.1)) == gd.ERR_INVALID
    assert call(sigma=0.0) == gd.ERR_INVALID
    assert call(lam=float("nan")) == gd.ERR_INVALID
    assert call(out=P(64)) == gd.ERR_INVALID  # aliasing
    o = gd.default_opts(fp64_refine=1)
    assert call(opts=ctypes.byref(o)) == gd.ERR_UNSUPPORTED
    assert lib.gd_npr_filter(P(64), 1, P(128), 1, 1 << 15, 1 << 14, 1, 0.001, 1.0, 1.0, 0.1, 1.25, 5.0, None, None,
                             None) == gd.ERR_UNSUPPORTED


def test_discretization_option_checked(lib):
    h = ctypes.c_void_p()
    o = gd.default_opts(discretization=3)
    assert lib.gd_hierarchy_create(ctypes.byref(h), 4, 4, 4, 0.1, 1.0, 1.0, 1.0, 1, ctypes.byref(o),
                                   None) == gd.ERR_INVALID
    assert lib.gd_smooth_z(P(64), 1, P(128), 1, 4, 4, 4, 1.0, 1.0, 4.0, ctypes.byref(o), None,
                           None) == gd.ERR_INVALID
    o = gd.default_opts(discretization=2, fp64_refine=1, storage=gd.F16)
    assert lib.gd_smooth_z(P(64), 1, P(128), 1, 4, 4, 4, 1.0, 1.0, 4.0, ctypes.byref(o), None,
                           None) == gd.ERR_UNSUPPORTED


def test_dct_argument_checks(lib):
    assert lib.gd_dct_solve(None, 0, P(64), 0, 8, 8, 8, 0.1, 1.0, 1.0, 1.0, None) == gd.ERR_INVALID
    assert lib.gd_dct_solve(P(64), 0, P(128), 0, 8, 8, 8, -0.1, 1.0, 1.0, 1.0, None) == gd.ERR_INVALID
    assert lib.gd_dct_solve(P(64), 0, P(128), 0, 6, 8, 8, 0.1, 1.0, 1.0, 1.0, None) == gd.ERR_UNSUPPORTED
    assert lib.gd_dct_solve(P(64), 0, P(128), 0, 8, 8, 8192, 0.1, 1.0, 1.0, 1.0, None) == gd.ERR_UNSUPPORTED
    assert lib.gd_dct_smooth_z(P(64), 1, P(128), 0, 8, 8, 8, 1.0, 1.0, 0.0, None) == gd.ERR_INVALID
    assert lib.gd_dct_smooth_z(P(64), 9, P(128), 0, 8, 8, 8, 1.0, 1.0, 4.0, None) == gd.ERR_INVALID


def test_plane_size_limit(lib):
    # an x-y plane above 2^28 cells is refused on the host, before any GPU call
    h = ctypes.c_void_p()
    assert lib.gd_hierarchy_create(ctypes.byref(h), 1 << 15, 1 << 14, 1, 0.1, 1.0, 1.0, 1.0, 1, None,
                                   None) == gd.ERR_UNSUPPORTED
    assert lib.gd_smooth_z(P(64), 1, P(128), 1, 1 << 15, 1 << 14, 2, 1.0, 1.0, 4.0, None, None,
                           None) == gd.ERR_UNSUPPORTED
    d = gd.make_slice_descs([0], 10, 10, 0.01, pitch=[(1 << 28) + 1])
    assert lib.gd_screened_poisson_slices(P(64), 1, P(128), 1, P(256), 1, d, 1, 1.0, 1.0, None, None, None,
                                          None) == gd.ERR_UNSUPPORTED


def test_step_argument_checks(lib):
    assert lib.gd_rb_sweep(P(64), P(64), P(128), 1, 4, 4, 4, 0.0, 1.0, 1.0, 1.0, None) == gd.ERR_INVALID
    assert lib.gd_residual_restrict(P(64), P(128), P(256), 1, 4, 4, 4, 3, 1, 1, 0.0, 1.0, 1.0, 1.0, None,
                                    None) == gd.ERR_INVALID
    assert lib.gd_prolong_add(P(64), P(128), 1, 4, 4, 4, 2, 2, 2, 5, None) == gd.ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.gd_hierarchy_create(ctypes.byref(h), 4, 4, 4, 0.0, 0.0, 0.0, 0.0, 1, None, None) == gd.ERR_INVALID
    assert lib.gd_hierarchy_create(ctypes.byref(h), 4, 4, 4, -1.0, 1.0, 0.0, 0.0, 1, None, None) == gd.ERR_INVALID


def test_streamed_hierarchy_argument_checks(lib):
    h = ctypes.c_void_p()
    o = gd.default_opts()
    create = lib.gd_hierarchy_create_streamed
    assert create(None, 8, 8, 8, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(o), 4, 0, None) == gd.ERR_INVALID
    assert create(ctypes.byref(h), 8, 8, 8, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(o), 0, 0, None) == gd.ERR_INVALID
    assert create(ctypes.byref(h), 8, 8, 8, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(o), 4, -1, None) == gd.ERR_INVALID
    assert create(ctypes.byref(h), 8, 8, 0, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(o), 4, 0, None) == gd.ERR_INVALID
    assert create(ctypes.byref(h), 8, 8, 8, 0.0, 0.0, 0.0, 0.0, 1, ctypes.byref(o), 4, 0, None) == gd.ERR_INVALID
    assert create(ctypes.byref(h), 8, 1, 8, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(o), 4, 0, None) == gd.ERR_UNSUPPORTED
    oh = gd.default_opts(discretization=1)
    assert create(ctypes.byref(h), 8, 8, 8, 0.0, 1.0, 1.0, 4.0, 1, ctypes.byref(oh), 4, 0, None) == gd.ERR_UNSUPPORTED
    assert not h.value
    assert lib.gd_vcycle_streamed(None, P(64), P(128), 1, None, None) == gd.ERR_INVALID
    assert lib.gd_hierarchy_device_bytes(None, None, None) == gd.ERR_INVALID
    assert lib.gd_hierarchy_streamed_levels(None, None) == gd.ERR_INVALID
    assert lib.gd_last_error()


def test_binding_refuses_out_of_bounds_slices():
    """The binding checks dtypes and that every slice lies inside each array
    before any call reaches the library (the kernels cannot see sizes)."""
    torch = pytest.importorskip("torch")
    d = gd.make_slice_descs([0, 100], 10, 10, 0.01)
    assert gd.slice_span(d) == 200
    assert gd.slice_span(gd.make_slice_descs([5], 4, 3, 0.01, pitch=[8])) == 5 + 8 * 2 + 4

    class Fake:  # a stand-in GPU tensor: the checks run before any pointer is used
        def __init__(self, n, dtype):
            self.shape, self.dtype, self.is_cuda, self._n = (n,), dtype, True, n

        def numel(self):
            return self._n

        def is_contiguous(self):
            return True

        def data_ptr(self):
            return 0

    ok, short = Fake(200, torch.float32), Fake(199, torch.float32)
    with pytest.raises(ValueError, match="reach"):
        gd.screened_poisson_slices(ok, Fake(200, torch.float32), d, out=short)
    with pytest.raises(ValueError, match="reach"):
        gd.screened_poisson_slices(short, Fake(199, torch.float32), d, out=ok)
    with pytest.raises(ValueError, match="I1"):
        gd.screened_poisson_slices(Fake(200, torch.float32), Fake(200, torch.float16), d, out=ok)
    with pytest.raises(ValueError, match="out_dtype"):
        gd.screened_poisson_slices(ok, Fake(200, torch.float32), d, out=Fake(200, torch.float16),
                                   out_dtype=torch.float32)


def test_binding_refuses_mismatched_hierarchy_arrays():
    torch = pytest.importorskip("torch")
    h = gd.Hierarchy.__new__(gd.Hierarchy)  # checks only: no library call is made
    h.shape, h.dtype, h._h = (4, 4, 4), torch.float32, None
    good = torch.zeros(4, 4, 4)
    with pytest.raises(ValueError):
        h.vcycle(torch.zeros(4, 4, 5), good)
    with pytest.raises(ValueError):
        h.vcycle(good.double(), good)
    with pytest.raises(ValueError):
        h.error_pairs(torch.zeros(2, 4, 4), good, 1)
    with pytest.raises(ValueError):
        h.rhs(torch.zeros(4, 4, 4, dtype=torch.float16))
    n = gd.Net.__new__(gd.Net)
    n._n = None
    with pytest.raises(ValueError):
        n.forward(torch.zeros(1, 4, 256, dtype=torch.float64))
    with pytest.raises(ValueError):
        n.train_step(torch.zeros(1, 4, 256), torch.zeros(1, 4, 128))


def test_net_create_takes_weights(lib):
    h = ctypes.c_void_p()
    w = (ctypes.c_float * 3)()
    # a wrong count is refused before any device work
    assert lib.gd_net_create(ctypes.byref(h), w, 3, 0) == gd.ERR_INVALID
    assert lib.gd_net_create(None, None, 0, 0) == gd.ERR_INVALID
