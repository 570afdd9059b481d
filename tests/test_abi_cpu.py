"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/dsrg_df.h declares, sizes workspaces, and
rejects every invalid argument before anything is enqueued."""
import ctypes
import os
import re

import pytest

from paper_1603_00561_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsrg_df.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dsrg_df_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(b.LIB_PATH):
        pytest.fail("libdsrgdf.so is not built; run python -m paper_1603_00561_amd.build")
    return b.load_library()


def test_exports_every_declared_function(lib):
    names = _declared_functions()
    assert set(names) >= {"dsrg_df_workspace_size", "dsrg_df_energy",
                          "dsrg_df_energy_backward", "dsrg_df_last_error"}
    for n in names:
        assert hasattr(lib, n), n
    assert set(b.EXPORTED) == set(names)
    assert lib.dsrg_df_version() >= 100


def _prob(nc=4, na=2, nv=70, naux=33, s=0.5, fake=True):
    # fake, aligned, non-null device addresses: never dereferenced because
    # every call below fails validation first
    a = 0x10000 if fake else None
    return b.Problem(nc, na, nv, naux, a, a, a, a, a, a, a, s)


def _ws(p, prec=0, terms=7, grad=0):
    out = ctypes.c_size_t(0)
    st = b.load_library().dsrg_df_workspace_size(ctypes.byref(p), prec, terms, grad, ctypes.byref(out))
    return st, out.value


def test_workspace_size_grows_with_problem(lib):
    st, small = _ws(_prob(4, 2, 70, 33))
    assert st == 0 and small > 0
    st, big = _ws(_prob(23, 6, 1100, 3000))
    assert st == 0
    # packed B_cv panels dominate: nc * ceil(nv/64)*64 * naux (rounded) doubles
    assert big >= 8 * 23 * 1152 * 3008
    st, cc = _ws(_prob(23, 6, 1100, 3000), terms=1)
    assert st == 0 and cc < big


@pytest.mark.parametrize("field,value,code", [
    ("nc", 0, b.DSRG_ERR_ARG), ("nv", 0, b.DSRG_ERR_ARG), ("naux", 0, b.DSRG_ERR_ARG),
    ("na", -1, b.DSRG_ERR_ARG), ("s", -0.1, b.DSRG_ERR_ARG), ("s", float("nan"), b.DSRG_ERR_ARG),
    ("s", float("inf"), b.DSRG_ERR_ARG), ("na", 9, b.DSRG_ERR_UNSUPPORTED),
])
def test_invalid_sizes_and_scalars(lib, field, value, code):
    p = _prob()
    setattr(p, field, value)
    st, _ = _ws(p)
    assert st == code
    assert lib.dsrg_df_last_error().decode()
    E = ctypes.c_void_p(0x20000)
    st = lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, ctypes.c_void_p(0x40000), 1 << 40, None)
    assert st == code


def test_slice_path_limits(lib):
    """Slice path: int32 level sums are exact up to naux = 33000; the
    gradient splits its longer contractions and has no such bound."""
    ok, _ = _ws(_prob(4, 2, 100, 33000), prec=2)
    assert ok == 0
    st, _ = _ws(_prob(4, 2, 100, 33001), prec=2)
    assert st == b.DSRG_ERR_UNSUPPORTED and "33000" in lib.dsrg_df_last_error().decode()
    assert _ws(_prob(4, 2, 100, 33001), prec=0)[0] == 0
    assert _ws(_prob(40, 2, 1100, 500), prec=2, grad=1)[0] == 0   # contraction 40*1152
    assert _ws(_prob(4, 2, 100, 64), prec=1)[0] == b.DSRG_ERR_UNSUPPORTED


def test_na_above_max_is_fine_for_ccvv_only(lib):
    p = _prob(na=20)
    st, _ = _ws(p, terms=1)
    assert st == 0


def test_bad_precision_and_terms(lib):
    p = _prob()
    assert _ws(p, prec=7)[0] == b.DSRG_ERR_ARG
    assert _ws(p, terms=0)[0] == b.DSRG_ERR_ARG
    assert _ws(p, terms=0x1000)[0] == b.DSRG_ERR_ARG
    assert _ws(p, terms=7 | b.OPT_ATOMIC_REDUCE)[0] == 0
    # the sign check bit is accepted and changes no workspace size
    assert _ws(p, terms=7 | b.OPT_CHECK_SIGNS) == _ws(p, terms=7)
    assert lib.dsrg_df_sign_check(None) == b.DSRG_ERR_ARG
    null = ctypes.POINTER(b.Problem)()
    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_workspace_size(null, 0, 7, 0, ctypes.byref(out)) == b.DSRG_ERR_ARG
    assert lib.dsrg_df_workspace_size(ctypes.byref(p), 0, 7, 0, None) == b.DSRG_ERR_ARG


def test_null_and_misaligned_pointers(lib):
    st, need = _ws(_prob())
    ws = ctypes.c_void_p(0x100000)
    E = ctypes.c_void_p(0x20000)
    for field in ("B_cv", "B_ca", "B_av", "eps_c", "eps_a", "eps_v", "gamma1"):
        for bad in (None, 0x10003):
            p = _prob()
            setattr(p, field, bad)
            st = lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, ws, need, None)
            assert st == b.DSRG_ERR_ARG, (field, bad)
            assert field in lib.dsrg_df_last_error().decode()
    # na == 0: active blocks may be NULL
    p = _prob(na=0)
    p.B_ca = p.B_av = p.eps_a = p.gamma1 = None
    # (not launched: workspace too small on purpose)
    st = lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, ws, 16, None)
    assert st == b.DSRG_ERR_WORKSPACE
    p = _prob()
    st = lib.dsrg_df_energy(ctypes.byref(p), 0, 7, None, ws, need, None)
    assert st == b.DSRG_ERR_ARG


def test_workspace_checks(lib):
    p = _prob()
    st, need = _ws(p)
    E = ctypes.c_void_p(0x20000)
    assert lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, ctypes.c_void_p(0x100000), need - 1,
                              None) == b.DSRG_ERR_WORKSPACE
    assert lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, None, need, None) == b.DSRG_ERR_WORKSPACE
    assert lib.dsrg_df_energy(ctypes.byref(p), 0, 7, E, ctypes.c_void_p(0x100008), need,
                              None) == b.DSRG_ERR_WORKSPACE


def test_last_error_is_cleared_by_a_good_call(lib):
    _ws(_prob(nc=0))
    assert lib.dsrg_df_last_error().decode()
    assert _ws(_prob())[0] == 0
    assert lib.dsrg_df_last_error().decode() == ""


def test_timing_filter_is_host_only_and_bounded(lib):
    # setting and clearing the filter touches no device; an over-long list is
    # refused and leaves the filter as it was
    assert lib.dsrg_df_timing_filter(b"ccvv_fp64,cavv_fp64_x") == 0
    assert lib.dsrg_df_timing_filter(b"x" * 300) == b.DSRG_ERR_ARG
    assert "255" in lib.dsrg_df_last_error().decode()
    assert lib.dsrg_df_timing_filter(b"") == 0
    assert lib.dsrg_df_timing_filter(None) == 0
    assert lib.dsrg_df_last_error().decode() == ""
    b.timing_filter(["ccvv_fp64"])
    b.timing_filter(None)
    with pytest.raises(b.DsrgError):
        b.timing_filter(["y" * 300])


def test_python_binding_refuses_cpu_tensors():
    import torch
    from paper_1603_00561_amd.workloads import make_problem
    p = make_problem(2, 1, 5, 8)
    t = [torch.from_numpy(x) for x in p.arrays()]
    with pytest.raises(ValueError, match="GPU"):
        b.energy(*t, p.s)


def _active(p, B_aa=0x30000, options=0, F=0x20000, ws=0x40000, ws_bytes=1 << 40):
    return b.load_library().dsrg_df_energy_active(
        ctypes.byref(p), ctypes.c_void_p(B_aa) if B_aa else None, options,
        ctypes.c_void_p(F) if F else None, ctypes.c_void_p(ws) if ws else None, ws_bytes, None)


def test_active_terms_entry_point_validation(lib):
    """F4-F8 entry point: workspace sizing and host-side rejection of every
    invalid argument (nothing is dereferenced or enqueued)."""
    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_active_workspace_size(ctypes.byref(_prob(23, 6, 1100, 3000)),
                                             ctypes.byref(out)) == 0
    # (xe|uf) for all active pairs dominates: na^2 (64 ceil(nv/64))^2 doubles
    assert out.value >= 8 * 36 * 1152 * 1152
    small = ctypes.c_size_t(0)
    assert lib.dsrg_df_active_workspace_size(ctypes.byref(_prob(23, 0, 1100, 3000)),
                                             ctypes.byref(small)) == 0
    assert 0 < small.value < 4096
    assert lib.dsrg_df_active_workspace_size(ctypes.byref(_prob()), None) == b.DSRG_ERR_ARG
    for field, value, code in (("nc", 0, b.DSRG_ERR_ARG), ("na", -1, b.DSRG_ERR_ARG),
                               ("s", float("nan"), b.DSRG_ERR_ARG),
                               ("na", 9, b.DSRG_ERR_UNSUPPORTED)):
        p = _prob()
        setattr(p, field, value)
        assert _active(p) == code, field
        assert lib.dsrg_df_last_error().decode()
    assert _active(_prob(), B_aa=0) == b.DSRG_ERR_ARG                  # B_aa missing
    assert _active(_prob(), B_aa=0x30004) == b.DSRG_ERR_ARG            # misaligned
    assert _active(_prob(), F=0) == b.DSRG_ERR_ARG
    assert _active(_prob(), options=0x100) == b.DSRG_ERR_ARG           # not an option here
    assert _active(_prob(), ws_bytes=16) == b.DSRG_ERR_WORKSPACE
    assert _active(_prob(), ws=0x40010) == b.DSRG_ERR_WORKSPACE        # not 256-aligned


def test_df_factors_entry_point_validation(lib):
    """DF-factor entry point: workspace sizing and host-side rejection."""
    def prob(**kw):
        d = dict(nao=40, nmo=40, naux=30, nfrz=2, nc=5, na=3, nv=30)
        d.update(kw)
        a = 0x10000
        return b.DFGenProblem(d["nao"], d["nmo"], d["naux"], d["nfrz"], d["nc"], d["na"],
                              d["nv"], a, a, a)

    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_factors_workspace_size(ctypes.byref(prob()), ctypes.byref(out)) == 0
    # at least the half-transformed integrals, naux (nc + na) nao doubles, the
    # transformed ones, naux (nc + na) (na + nv), and three naux x naux metrics
    assert out.value >= 8 * (30 * 8 * 40 + 30 * 8 * 33 + 3 * 30 * 30)

    def call(p, B=(0x20000, 0x20000, 0x20000, 0x20000), opts=0, ws=0x40000, nb=1 << 40):
        return lib.dsrg_df_factors(ctypes.byref(p), opts,
                                   *[ctypes.c_void_p(x) if x else None for x in B],
                                   ctypes.c_void_p(ws) if ws else None, nb, None)

    for kw in (dict(nao=0), dict(naux=0), dict(nc=0), dict(nv=0), dict(na=-1),
               dict(nmo=39)):
        assert call(prob(**kw)) == b.DSRG_ERR_ARG, kw
        assert lib.dsrg_df_last_error().decode()
    assert call(prob(), B=(0, 0x20000, 0x20000, 0x20000)) == b.DSRG_ERR_ARG
    assert call(prob(), B=(0x20000, 0, 0x20000, 0x20000)) == b.DSRG_ERR_ARG
    assert call(prob(), opts=0x100) == b.DSRG_ERR_ARG
    assert call(prob(), nb=16) == b.DSRG_ERR_WORKSPACE
    assert call(prob(), ws=0x40008) == b.DSRG_ERR_WORKSPACE


def test_fock_entry_point_validation(lib):
    """Generalized-Fock entry point: workspace sizing and host-side rejection
    (no device work is launched: every call fails before the first launch)."""
    def prob(h=0x10000, g1=0x10000, **kw):
        d = dict(nao=40, nmo=40, naux=30, nfrz=2, nc=5, na=3, nv=30)
        d.update(kw)
        a = 0x10000
        return b.FockProblem(b.DFGenProblem(d["nao"], d["nmo"], d["naux"], d["nfrz"], d["nc"],
                                            d["na"], d["nv"], a, a, a), h, g1)

    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_fock_workspace_size(ctypes.byref(prob()), ctypes.byref(out)) == 0
    # at least the occupied-row integrals and factors, (10 occupied) x 40 MOs
    # per auxiliary function, three of them, and three naux x naux metrics
    assert out.value >= 8 * (3 * 30 * 10 * 40 + 3 * 30 * 30)
    assert lib.dsrg_df_fock_workspace_size(None, ctypes.byref(out)) == b.DSRG_ERR_ARG

    def call(p, F=0x20000, opts=0, ws=0x40000, nb=1 << 40):
        return lib.dsrg_df_fock(ctypes.byref(p), opts, ctypes.c_void_p(F) if F else None,
                                ctypes.c_void_p(ws) if ws else None, nb, None)

    for kw in (dict(nao=0), dict(naux=0), dict(nc=0), dict(nv=0), dict(na=-1), dict(nmo=39)):
        assert call(prob(**kw)) == b.DSRG_ERR_ARG, kw
        assert lib.dsrg_df_last_error().decode()
    assert call(prob(h=0)) == b.DSRG_ERR_ARG
    assert call(prob(g1=0)) == b.DSRG_ERR_ARG            # na > 0 needs gamma1
    assert call(prob(g1=0x10004)) == b.DSRG_ERR_ARG      # misaligned
    assert call(prob(), F=0) == b.DSRG_ERR_ARG
    assert call(prob(), opts=0x100) == b.DSRG_ERR_ARG
    assert call(prob(), nb=16) == b.DSRG_ERR_WORKSPACE
    assert call(prob(), ws=0x40008) == b.DSRG_ERR_WORKSPACE


def test_semicanonicalize_entry_point_validation(lib):
    """Semicanonicalization entry point: workspace sizing and host-side
    rejection (every call below fails before the first launch)."""
    def prob(F=0x10000, C=0, **kw):
        d = dict(nao=0, nmo=40, nfrz=2, nc=5, na=3, nv=30)
        d.update(kw)
        return b.SemicanProblem(d["nao"], d["nmo"], d["nfrz"], d["nc"], d["na"], d["nv"], F, C)

    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_semicanonicalize_workspace_size(ctypes.byref(prob()),
                                                       ctypes.byref(out)) == 0
    # three padded 32 x 32 Jacobi matrices at least
    assert out.value >= 3 * 8 * 32 * 32

    def call(p, U=0x20000, eps=0x30000, Cs=0, opts=0, ws=0x40000, nb=1 << 40, info=0):
        v = lambda x: ctypes.c_void_p(x) if x else None  # noqa: E731
        return lib.dsrg_df_semicanonicalize(ctypes.byref(p), opts, v(U), v(eps), v(Cs), v(info),
                                            v(ws), nb, None)

    for kw in (dict(nmo=0), dict(nc=-1), dict(nmo=39)):
        assert call(prob(**kw)) == b.DSRG_ERR_ARG, kw
        assert lib.dsrg_df_last_error().decode()
    assert call(prob(F=0)) == b.DSRG_ERR_ARG
    assert call(prob(), U=0) == b.DSRG_ERR_ARG
    assert call(prob(), eps=0x30004) == b.DSRG_ERR_ARG
    assert call(prob(), info=0x50002) == b.DSRG_ERR_ARG   # info must be 4-byte aligned
    assert call(prob(), Cs=0x50000) == b.DSRG_ERR_ARG                  # Cs without C
    assert call(prob(C=0x50000, nao=40)) == b.DSRG_ERR_ARG             # C without Cs
    assert call(prob(), opts=0x100) == b.DSRG_ERR_ARG
    assert call(prob(), nb=16) == b.DSRG_ERR_WORKSPACE
    assert call(prob(), ws=0x40008) == b.DSRG_ERR_WORKSPACE


def test_cholesky_entry_point_validation(lib):
    """CD-factor entry point: workspace sizing and host-side rejection (every
    call below fails before the first launch)."""
    def prob(nao=20, M=0x10000, tol=1e-5, max_rank=50):
        return b.CDProblem(nao, M, tol, max_rank)

    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_cholesky_workspace_size(ctypes.byref(prob()), ctypes.byref(out)) == 0
    # at least the residual diagonal over the 210 pairs
    assert out.value >= 8 * 210
    assert b.cholesky_workspace_size(20, 50) == out.value

    def call(p, B=0x20000, rank=0x30000, dmax=0x30100, piv=0x30200, opts=0, ws=0x40000,
             nb=1 << 40):
        v = lambda x: ctypes.c_void_p(x) if x else None
        return lib.dsrg_df_cholesky(ctypes.byref(p), opts, v(B), v(rank), v(dmax), v(piv), v(ws),
                                    nb, None)

    for kw in (dict(nao=0), dict(tol=-1.0), dict(tol=float("nan")), dict(tol=float("inf")),
               dict(max_rank=-1), dict(max_rank=211)):
        assert call(prob(**kw)) == b.DSRG_ERR_ARG, kw
        assert lib.dsrg_df_last_error().decode()
    assert call(prob(nao=b_max_nao() + 1)) == b.DSRG_ERR_UNSUPPORTED
    assert call(prob(M=0)) == b.DSRG_ERR_ARG
    assert call(prob(M=0x10004)) == b.DSRG_ERR_ARG                    # misaligned
    assert call(prob(), B=0) == b.DSRG_ERR_ARG
    assert call(prob(), rank=0) == b.DSRG_ERR_ARG
    assert call(prob(), dmax=0) == b.DSRG_ERR_ARG
    assert call(prob(), piv=0x30204) == b.DSRG_ERR_ARG                # optional, but aligned
    assert call(prob(), opts=0x100) == b.DSRG_ERR_ARG
    assert call(prob(), nb=16) == b.DSRG_ERR_WORKSPACE
    assert call(prob(), ws=0x40008) == b.DSRG_ERR_WORKSPACE
    assert call(prob(), ws=0) == b.DSRG_ERR_WORKSPACE


def b_max_nao():
    text = open(HEADER).read()
    return int(re.search(r"#define DSRG_CD_MAX_NAO (\d+)", text).group(1))


def test_factor_build_without_metric_sizes(lib):
    """J = NULL (CD vectors in ao3): smaller workspaces, same validation."""
    assert b.df_factors_workspace_size(40, 40, 30, 2, 5, 3, 30, metric=False) < \
        b.df_factors_workspace_size(40, 40, 30, 2, 5, 3, 30)
    assert b.df_fock_workspace_size(40, 40, 30, 2, 5, 3, 30, metric=False) < \
        b.df_fock_workspace_size(40, 40, 30, 2, 5, 3, 30)
    a = 0x10000
    p = b.DFGenProblem(40, 40, 30, 2, 5, 3, 30, a, ctypes.c_void_p(0x10004), a)
    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_factors_workspace_size(ctypes.byref(p), ctypes.byref(out)) == 0
    st = lib.dsrg_df_factors(ctypes.byref(p), 0, *[ctypes.c_void_p(0x20000)] * 4,
                             ctypes.c_void_p(0x40000), 1 << 40, None)
    assert st == b.DSRG_ERR_ARG                                        # misaligned J


def test_laplace_fit_matches_the_oracle_and_validates(lib):
    """The library's host fit (Householder QR) against the oracle's (numpy
    least squares): the same exponents, the same largest error, the same
    fitted function; and the host-side rejection of bad arguments."""
    import numpy as np
    from oracle import dsrg_laplace as L
    for s, nq in ((0.5, 8), (0.5, 16), (1.0, 12), (1e8, 10), (0.0, 4), (0.3, 1)):
        t, w, err = b.laplace_fit(s, 0.8, 14.0, nq)
        to, wo, eo = L.laplace_fit(s, 0.8, 14.0, nq)
        assert np.allclose(t, to, rtol=1e-14, atol=0)
        assert err == pytest.approx(eo, rel=1e-6, abs=1e-300)
        xc = np.geomspace(0.8, 14.0, 2000)
        f = np.exp(-np.outer(xc, t)) @ w
        fo = np.exp(-np.outer(xc, to)) @ wo
        assert np.abs(f - fo).max() <= max(1e-3 * eo, 1e-14)
    d = ctypes.POINTER(ctypes.c_double)
    buf = (ctypes.c_double * 64)()
    e = ctypes.c_double(0.0)
    for args in ((-1.0, 0.8, 14.0, 4), (0.5, 0.0, 14.0, 4), (0.5, 2.0, 1.0, 4),
                 (0.5, 0.8, 14.0, 0), (0.5, 0.8, 14.0, 65), (float("nan"), 0.8, 14.0, 4)):
        assert lib.dsrg_df_laplace_fit(*args, buf, buf, ctypes.byref(e)) == b.DSRG_ERR_ARG, args
    assert lib.dsrg_df_laplace_fit(0.5, 0.8, 14.0, 4, None, buf, ctypes.byref(e)) == b.DSRG_ERR_ARG


def test_coulomb_laplace_entry_point_validation(lib):
    import numpy as np
    p = _prob(nc=4, na=0, nv=30, naux=20)
    out = ctypes.c_size_t(0)
    assert lib.dsrg_df_laplace_workspace_size(ctypes.byref(p), 8, ctypes.byref(out)) == 0
    assert out.value >= 8 * (20 * 4 * 30 + 20 * 20)
    for nq in (0, 65):
        assert lib.dsrg_df_laplace_workspace_size(ctypes.byref(p), nq, ctypes.byref(out)) == \
            b.DSRG_ERR_ARG
    d = ctypes.POINTER(ctypes.c_double)
    t = np.array([0.1, 1.0, 3.0])
    w = np.array([1.0, -0.5, 0.25])

    def call(p, t=t, w=w, opts=0, E=0x20000, S=0, ws=0x40000, nb=1 << 40):
        v = lambda x: ctypes.c_void_p(x) if x else None
        return lib.dsrg_df_coulomb_laplace(ctypes.byref(p), len(t), t.ctypes.data_as(d),
                                           w.ctypes.data_as(d), opts, v(E), v(S), v(ws), nb, None)

    assert call(_prob(nc=0, na=0, nv=30, naux=20)) == b.DSRG_ERR_ARG
    assert call(p, t=np.array([0.1, 0.0, 3.0])) == b.DSRG_ERR_ARG        # t must be > 0
    assert call(p, w=np.array([1.0, float("inf"), 0.0])) == b.DSRG_ERR_ARG
    assert call(p, E=0) == b.DSRG_ERR_ARG
    assert call(p, S=0x20004) == b.DSRG_ERR_ARG                           # misaligned
    assert call(p, opts=0x100) == b.DSRG_ERR_ARG
    assert call(p, nb=16) == b.DSRG_ERR_WORKSPACE
    assert call(p, ws=0x40008) == b.DSRG_ERR_WORKSPACE


def test_mfma_probe_validation(lib):
    v = ctypes.c_void_p
    good = dict(kind=0, nwg=256, iters=16, stamps=0x10000, sink=0x20000)

    def call(**kw):
        a = dict(good, **kw)
        return lib.dsrg_df_mfma_probe(a["kind"], a["nwg"], a["iters"],
                                      v(a["stamps"]) if a["stamps"] else None,
                                      v(a["sink"]) if a["sink"] else None, None)

    for bad in (dict(kind=2), dict(kind=-1), dict(nwg=0), dict(nwg=65537), dict(iters=0),
                dict(iters=(1 << 24) + 1), dict(stamps=0), dict(sink=0), dict(stamps=0x10004),
                dict(sink=0x20004)):
        assert call(**bad) == b.DSRG_ERR_ARG, bad
        assert lib.dsrg_df_last_error()
