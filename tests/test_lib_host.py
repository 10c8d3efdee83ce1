"""Host-side checks of libfdlb (no GPU needed): the shared library loads and exports
every entry point include/fdlb.h declares, its quadrature agrees with the oracle's
independent construction, and problem set-up validates inputs and computes the
same time step as the oracle."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


@pytest.fixture(scope="module")
def F():
    import paper_1308_0692_amd as F
    return F


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(fdlb\w+)\s*\(", src, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    assert "fdlb_step" in names and "fdlb_solve_steady" in names
    assert len(names) > 25


def test_library_exports_every_declared_symbol(F):
    lib = C.CDLL(F._lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_half_range_matches_oracle(F, n):
    from oracle import quadrature as q
    x, w = F.quad_half_range(n)
    xo, wo = q.half_range(n)
    assert np.allclose(x, xo, rtol=4e-16, atol=0)
    assert np.allclose(w, wo, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12, 20, 32])
def test_full_range_matches_oracle(F, n):
    from oracle import quadrature as q
    x, w = F.quad_full_range(n)
    xo, wo = q.full_range(n)
    assert np.allclose(x, xo, rtol=1e-15, atol=1e-300)
    assert np.allclose(w, wo, rtol=1e-14, atol=0)
    if n % 2:
        assert x[n // 2] == 0.0


def test_quadrature_rejects_bad_orders(F):
    x = np.empty(80)
    for n in (0, 17, -3):
        assert F._lib.lib.fdlb_quad_half_range(n, F._lib._dp(x), F._lib._dp(x)) == F._lib.EINVAL
    assert F._lib.lib.fdlb_quad_half_range(2, None, None) == F._lib.EINVAL
    assert F._lib.lib.fdlb_quad_full_range(33, F._lib._dp(x), F._lib._dp(x)) == F._lib.EINVAL


@pytest.mark.parametrize("case", [W.C1, W.C2, W.C4, W.couette_x(50), W.cavity(37, ny=29, order=3),
                                  W.cavity(64, kn=float("inf"), order=2),
                                  W.with_(W.cavity(40, ny=20, order=2), lx=2.0, ly=1.0),
                                  W.with_(W.couette(50), ly=0.3)])
def test_time_step_and_velocities_match_oracle(F, case):
    from oracle.scheme import Problem as OP
    p = F.Problem(case, bind=False)
    o = OP.from_case(case)
    assert p.q == o.q
    assert p.dt == pytest.approx(o.dt, rel=1e-15)
    assert p.omega == pytest.approx(o.omega, rel=1e-15, abs=0)
    x, y, w = p.velocities()
    assert np.allclose(x, o.xi_x, rtol=1e-15, atol=0)
    assert np.allclose(y, o.xi_y, rtol=1e-15, atol=0)
    assert np.allclose(w, o.w, rtol=1e-15, atol=0)


def test_sizes(F):
    p = F.Problem(W.C4, bind=False)
    assert p.state_bytes == 2 * 256 * 1024 * 1024 * 4
    assert p.workspace_bytes < 128 * 2 ** 20   # FP64 moments (48 MB) + staging (32 MB) for 1024^2
    p = F.Problem(W.C1, bind=False)
    assert p.state_bytes == 2 * ((24 * 200 * 8 + 255) // 256 * 256)


def test_validation_errors(F):
    bad = [W.with_(W.C2, nx=0), W.with_(W.C2, periodic_x=True),
           W.with_(W.C2, cfl=-1.0), W.with_(W.C2, kn=0.0), W.with_(W.C2, qx=("half", 17)),
           W.with_(W.C2, qy=("full", 0)), W.with_(W.C2, nx=1)]
    for c in bad:
        with pytest.raises(F.FdlbError) as e:
            F.Problem(c, bind=False)
        assert e.value.code == F._lib.EINVAL, c
    # stability limits of the explicit scheme
    for c in (W.with_(W.C2, kn=0.001), W.with_(W.C2, cfl=1.2)):
        with pytest.raises(F.FdlbError) as e:
            F.Problem(c, bind=False)
        assert e.value.code == F._lib.EUNSTABLE
        F.Problem(c, bind=False, allow_unstable=True)


def test_calls_before_bind_are_state_errors(F):
    p = F.Problem(W.C2, bind=False)
    assert F._lib.lib.fdlb_step(p._h, 1) == F._lib.ESTATE
    assert "bind" in F._lib.lib.fdlb_last_error().decode()
    assert F._lib.lib.fdlb_step(None, 1) == F._lib.EINVAL


def test_tiles_listed_and_heuristic_fits(F):
    for prec in ("fp32", "fp64"):
        n = F.tile_count(prec)
        assert n >= 6
        for t in range(n):
            assert "vx" in F.tile_describe(prec, t)
    for case in (W.C1, W.C2, W.C4, W.cavity(2, kn=1.0, order=2), W.cavity(37, ny=29), W.couette_x(40)):
        for prec in ("fp32", "fp64"):
            p = F.Problem(case, precision=prec, bind=False)
            assert 0 <= p.tile < F.tile_count(prec)


def test_mixed_precision_problem_sizes(F):
    """A mixed-precision problem is sized for double and starts in float (host only)."""
    case = W.cavity(48, kn=0.2, order=2)
    m = F.Problem(case, precision="mixed", bind=False)
    d = F.Problem(case, precision="fp64", bind=False)
    s = F.Problem(case, precision="fp32", bind=False)
    assert m.state_bytes == d.state_bytes == 2 * s.state_bytes
    assert F._lib.lib.fdlb_problem_active_precision(m._h) == F._lib.FP32
    assert F._lib.lib.fdlb_problem_active_precision(d._h) == F._lib.FP64
    # switching needs a bound, seeded state
    assert F._lib.lib.fdlb_promote(m._h) == F._lib.ESTATE
    assert F._lib.lib.fdlb_promote(s._h) == F._lib.ESTATE


def _mlp(F, hidden=4, max_batch=512):
    h = C.c_void_p()
    assert F._lib.lib.fdlb_mlp_create(hidden, max_batch, C.byref(h)) == 0
    return h


def test_network_layout_and_initialisation(F):
    """Parameter count and layout of the warm-start network, Glorot bounds, zero biases and a
    deterministic stream per seed (host only)."""
    from oracle import mlp
    lib = F._lib.lib
    for hidden in (1, 2, 4, 8):
        h = _mlp(F, hidden)
        P = lib.fdlb_mlp_param_count(h)
        assert P == mlp.param_count(128, hidden)
        p1 = np.empty(P, dtype=np.float32)
        p2 = np.empty(P, dtype=np.float32)
        p3 = np.empty(P, dtype=np.float32)
        fp = C.POINTER(C.c_float)
        assert lib.fdlb_mlp_init_params(h, 5, p1.ctypes.data_as(fp)) == 0
        assert lib.fdlb_mlp_init_params(h, 5, p2.ctypes.data_as(fp)) == 0
        assert lib.fdlb_mlp_init_params(h, 6, p3.ctypes.data_as(fp)) == 0
        assert np.array_equal(p1, p2) and not np.array_equal(p1, p3)
        for (Wm, b), (o, i) in zip(mlp.unpack(p1.astype(np.float64), 128, hidden), mlp.layer_shapes(128, hidden)):
            lim = math.sqrt(6.0 / (o + i))
            assert np.abs(Wm).max() <= lim and np.abs(Wm).max() > 0.9 * lim
            assert abs(Wm.mean()) < 0.1 * lim
            assert np.all(b == 0)
        assert lib.fdlb_mlp_workspace_bytes(h) > 0
        lib.fdlb_mlp_destroy(h)


def test_network_argument_errors(F):
    lib = F._lib.lib
    h = C.c_void_p()
    assert lib.fdlb_mlp_create(0, 512, C.byref(h)) == F._lib.EINVAL
    assert lib.fdlb_mlp_create(9, 512, C.byref(h)) == F._lib.EINVAL
    assert lib.fdlb_mlp_create(4, 0, C.byref(h)) == F._lib.EINVAL
    h = _mlp(F)
    assert lib.fdlb_mlp_forward(h, None, 0, None) == F._lib.ESTATE   # not bound
    assert lib.fdlb_mlp_adam_step(h, 1e-3, 0.9, 0.999, 1e-8, 1) == F._lib.ESTATE
    assert lib.fdlb_mlp_param_count(None) == F._lib.EINVAL
    lib.fdlb_mlp_destroy(h)


def test_domain_lengths_default_and_validation(F):
    """lx = ly = 0 in a description mean the unit length; negative or non-finite lengths are
    rejected (host only)."""
    case = W.cavity(32, order=2)
    d0 = F._lib.desc_from_case(case)
    d0.lx = d0.ly = 0.0
    p0 = F.Problem(desc=d0, bind=False)
    p1 = F.Problem(case, bind=False)
    assert p0.dt == p1.dt
    for bad in (-1.0, float("inf"), float("nan")):
        d = F._lib.desc_from_case(case)
        d.lx = bad
        with pytest.raises(F.FdlbError) as e:
            F.Problem(desc=d, bind=False)
        assert e.value.code == F._lib.EINVAL


def test_kernel_resource_report_parser():
    from paper_1308_0692_amd import build as B
    text = """k.hip:9:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]
    9 | __global__ void foo(float* p) {}
      | ^
k.hip:9:1: remark:     SGPRs: 18 [-Rpass-analysis=kernel-resource-usage]
k.hip:9:1: remark:     VGPRs: 59 [-Rpass-analysis=kernel-resource-usage]
k.hip:9:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:9:1: remark:     ScratchSize [bytes/lane]: 12 [-Rpass-analysis=kernel-resource-usage]
k.hip:9:1: remark:     Occupancy [waves/SIMD]: 8 [-Rpass-analysis=kernel-resource-usage]
k.hip:9:1: remark:     LDS Size [bytes/block]: 0 [-Rpass-analysis=kernel-resource-usage]
"""
    r = B.parse_resources(text)
    assert r == {"_Z3fooPf": {"sgpr": 18, "vgpr": 59, "agpr": 0, "scratch": 12, "waves_per_simd": 8, "lds": 0}}


def test_built_step_kernels_use_no_scratch():
    """The build's resource report (written next to the objects): no step kernel spills or keeps
    a stack copy, and every one fits at least one wave per SIMD."""
    import json
    import os
    from paper_1308_0692_amd import build as B
    path = os.path.join(B.BUILD, "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("no build report (library built elsewhere)")
    rep = json.load(open(path))
    steps = {k: v for k, v in rep.items() if "step_kernel" in k}
    assert steps
    assert all(v.get("scratch", 0) == 0 for v in steps.values())
    assert all(v.get("waves_per_simd", 0) >= 1 for v in steps.values())


def test_batch_reports_each_members_velocity_count():
    """A batch is created on the host alone; each member's Q comes from its own velocity sets,
    and an index out of range is an error."""
    from paper_1308_0692_amd import _lib
    descs = [_lib.make_desc(32, 32, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, ("half", 2), ("half", 2)),
             _lib.make_desc(40, 40, False, False, (0.0, 0.01, 0.0, 0.0), 1.0, ("half", 4), ("half", 3)),
             _lib.make_desc(24, 16, False, False, (0.0, 0.01, 0.0, 0.0), 0.3, ("half", 3), ("half", 4))]
    for d in descs:
        d.precision = _lib.PRECISIONS["fp32"]
    arr = (_lib.ProblemDesc * len(descs))(*descs)
    h = C.c_void_p()
    assert _lib.lib.fdlb_batch_create(arr, len(descs), C.byref(h)) == 0
    try:
        assert [_lib.lib.fdlb_batch_problem_q(h, i) for i in range(3)] == [16, 48, 48]
        assert _lib.lib.fdlb_batch_problem_q(h, 3) == _lib.EINVAL
        assert _lib.lib.fdlb_batch_problem_q(h, -1) == _lib.EINVAL
    finally:
        _lib.lib.fdlb_batch_destroy(h)


def test_batch_create_rejects_bad_arguments(F):
    """No problems, a NULL description array or output, mixed precisions, and an invalid member
    (named in the message) are errors, and no handle is returned."""
    from paper_1308_0692_amd import _lib
    good = _lib.make_desc(32, 32, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, ("half", 2), ("half", 2))
    bad = _lib.make_desc(0, 32, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, ("half", 2), ("half", 2))
    other = _lib.make_desc(32, 32, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, ("half", 2), ("half", 2),
                           precision="fp64")
    h = C.c_void_p()
    one = (_lib.ProblemDesc * 1)(good)
    assert _lib.lib.fdlb_batch_create(one, 0, C.byref(h)) == _lib.EINVAL and not h.value
    assert _lib.lib.fdlb_batch_create(None, 1, C.byref(h)) == _lib.EINVAL and not h.value
    assert _lib.lib.fdlb_batch_create(one, 1, None) == _lib.EINVAL
    assert _lib.lib.fdlb_batch_create((_lib.ProblemDesc * 2)(good, other), 2, C.byref(h)) == _lib.EINVAL
    assert not h.value and b"precision" in _lib.lib.fdlb_last_error()
    assert _lib.lib.fdlb_batch_create((_lib.ProblemDesc * 2)(good, bad), 2, C.byref(h)) == _lib.EINVAL
    assert not h.value and _lib.lib.fdlb_last_error().startswith(b"problem 1:")


def test_builtin_tile_choices_of_the_workloads(F):
    """The built-in shape choices that the measured results rest on: single-cell-wide channels
    take the 64-cell column split eight ways, small cavities the 64 x 1 tile split eight ways
    (latency-bound), the large cavity a wide non-temporal tile without a split (bandwidth-bound);
    and no shape is compiled twice."""
    for prec in ("fp32", "fp64"):
        descs = [F.tile_describe(prec, t) for t in range(F.tile_count(prec))]
        assert len(set(descs)) == len(descs), prec
        for case in (W.C1, W.couette(37)):
            assert F.tile_describe(prec, F.Problem(case, precision=prec, bind=False).tile) == "vx1 lx1 k1 w1 a8 (1x64)"
        assert F.tile_describe(prec, F.Problem(W.C2, precision=prec, bind=False).tile) == "vx1 lx64 k1 w1 a8 (64x1)"
        big = F.tile_describe(prec, F.Problem(W.C4, precision=prec, bind=False).tile)
        assert " nt " in big and " a" not in big and big.startswith("vx4" if prec == "fp32" else "vx2"), big


def test_problems_created_from_many_threads_at_once(F):
    """Distinct handles are independent: problems created concurrently from eight threads (their
    quadrature rules overlapping, so the rule cache is shared) give the same velocity sets and
    time steps as problems created alone, and each thread's error message stays its own."""
    import threading
    from paper_1308_0692_amd import _lib
    orders = [2, 3, 4, 5, 6, 7, 8, 3]
    bad = _lib.make_desc(0, 8, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, ("half", 2), ("half", 2))

    def make(order):
        d = _lib.make_desc(16, 12, False, False, (0.0, 0.01, 0.0, 0.0), 0.3, ("half", order), ("half", order + 1))
        h = C.c_void_p()
        assert _lib.lib.fdlb_problem_create(C.byref(d), C.byref(h)) == 0
        q = _lib.lib.fdlb_problem_q(h)
        x, y, w = (np.empty(q) for _ in range(3))
        assert _lib.lib.fdlb_problem_velocities(h, *[_lib._dp(a) for a in (x, y, w)]) == 0
        dt = _lib.lib.fdlb_problem_dt(h)
        _lib.lib.fdlb_problem_destroy(h)
        return q, dt, x, y, w

    alone = {o: make(o) for o in set(orders)}
    errors, results = [], []

    def work(order):
        try:
            for _ in range(20):
                got = make(order)
                ref = alone[order]
                assert got[0] == ref[0] and got[1] == ref[1]
                assert all(np.array_equal(a, b) for a, b in zip(got[2:], ref[2:]))
                h = C.c_void_p()
                assert _lib.lib.fdlb_problem_create(C.byref(bad), C.byref(h)) == _lib.EINVAL
                assert _lib.lib.fdlb_last_error() == b"nx and ny must be >= 1"
                make(order)  # a success clears this thread's message
                assert _lib.lib.fdlb_last_error() == b""
            results.append(order)
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(o,)) for o in orders]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    assert sorted(results) == sorted(orders)


def test_full_range_rule_on_a_bounded_axis_is_accepted(F):
    """Walls take either kind of rule on their normal axis: Eq. (9) read as impermeability
    divides by the rule's own leaving flux (the standard lattice D2Q16 is 4 x 4 full-range
    nodes).  The time step follows the rule's largest speed as for half-range sets."""
    from paper_1308_0692_amd import _lib
    for qx, qy in ((("full", 4), ("half", 4)), (("half", 4), ("full", 3)), (("full", 4), ("full", 4)),
                   (("full", 5), ("full", 6))):
        d = _lib.make_desc(16, 16, False, False, (0.0, 0.01, 0.0, 0.0), 0.1, qx, qy)
        h = C.c_void_p()
        assert _lib.lib.fdlb_problem_create(C.byref(d), C.byref(h)) == _lib.OK, (qx, qy)
        xs, _ = _lib.quad_full_range(qx[1]) if qx[0] == "full" else _lib.quad_half_range(qx[1])
        ys, _ = _lib.quad_full_range(qy[1]) if qy[0] == "full" else _lib.quad_half_range(qy[1])
        assert _lib.lib.fdlb_problem_dt(h) == pytest.approx(0.9 / (16 * (np.abs(xs).max() + np.abs(ys).max())),
                                                            rel=1e-15)
        _lib.lib.fdlb_problem_destroy(h)
    for case in (W.C1, W.couette_x(40, qy=("full", 3)), W.couette(30, qx=("full", 2))):
        assert F.Problem(case, bind=False).q > 0


def test_one_node_rules_are_rejected(F):
    """A rule must integrate xi^2 exactly for the relaxation to conserve momentum: one node per
    half-line (sum w xi^2 = 2/pi) and the one-node full-range rule (xi = 0) are rejected, two
    nodes are accepted; the quadrature routines themselves still give the one-node rules."""
    from paper_1308_0692_amd import _lib
    for case in (W.cavity(12, order=1), W.couette(20, qx=("full", 1)), W.couette(20, qy=("half", 1))):
        with pytest.raises(F.FdlbError) as e:
            F.Problem(case, bind=False)
        assert e.value.code == _lib.EINVAL and "at least 2 nodes" in str(e.value)
    assert F.Problem(W.cavity(12, order=2), bind=False).q == 16
    assert F.Problem(W.couette(20, qx=("full", 2), qy=("half", 2)), bind=False).q == 8
    x, w = _lib.quad_half_range(1)
    assert np.allclose(x, [-np.sqrt(2 / np.pi), np.sqrt(2 / np.pi)]) and np.allclose(w, [0.5, 0.5])
    assert abs(float(np.sum(w * x * x)) - 2 / np.pi) < 1e-15


def test_pseudo_time_stretches_follow_their_definition(F):
    """s_alpha = max(1, min(cfl / (nu_alpha (1 - omega) + omega / 2), 1 / omega, 64)) with nu_alpha
    the velocity's own Courant number over the bounded axes."""
    for case in (W.cavity(48, kn=0.05, order=4), W.cavity(20, ny=12, kn=3.0, order=6),
                 W.couette(40, kn=float("inf"), qy=("half", 8)),
                 W.with_(W.cavity(16, kn=0.2), qx=("full", 5), qy=("full", 5))):
        p = F.Problem(case, precision="fp64", bind=False)
        x, y, w = p.velocities()
        nu = p.dt * (np.abs(x) * (0 if case.periodic_x else case.nx) + np.abs(y) * (0 if case.periodic_y else case.ny))
        want = np.full(p.q, 64.0)
        den = nu * (1.0 - p.omega) + 0.5 * p.omega
        want = np.where(den > 0, np.minimum(want, case.cfl / np.where(den > 0, den, 1)), want)
        if p.omega > 0:
            want = np.minimum(want, 1.0 / p.omega)
        else:
            want = np.where(nu == 0, 1.0, want)
        want = np.maximum(want, 1.0)
        assert np.array_equal(p.pseudo_weights(), want.astype(np.float32).astype(np.float64)), case.name
        # the problem's margin: s (omega + 2 nu (1 - omega)) <= 2 cfl, s omega <= 1
        s = p.pseudo_weights()
        assert np.all(s * (p.omega + 2 * nu * (1 - p.omega)) <= 2 * case.cfl * (1 + 1e-6) + 1e-12)
        assert np.all(s * p.omega <= 1 + 1e-6)


def _hybrid_create(F, descs):
    L = F._lib
    arr = (L.HybridDesc * len(descs))(*descs)
    h = C.c_void_p()
    code = L.lib.fdlb_hybrid_create(arr, len(descs), C.byref(h))
    return code, h


def test_hybrid_layout_time_step_and_errors(F):
    """Host side of the hybrid channel: time step and omega equal the oracle's to the last bit,
    the state holds 2 layer Q_layer + (ny - 2 layer) Q_bulk doubles, bad descriptions are
    refused, and calls before binding are state errors."""
    from oracle.hybrid import HybridChannel
    L = F._lib
    cases = [(200, 40, 0.1, 4, 4, ("full", 3)), (37, 1, 0.05, 4, 3, ("full", 3)), (30, 15, 0.2, 3, 3, ("half", 2)),
             (64, 12, math.inf, 2, 7, ("full", 2))]
    descs = [L.make_hybrid_desc(ny, lay, kn, (-0.01, 0.01), nh, nf, qx) for ny, lay, kn, nh, nf, qx in cases]
    code, h = _hybrid_create(F, descs)
    assert code == 0
    total = 0
    for i, (ny, lay, kn, nh, nf, qx) in enumerate(cases):
        ql, qb, sd = C.c_int32(), C.c_int32(), C.c_int64()
        dt, om = C.c_double(), C.c_double()
        assert L.lib.fdlb_hybrid_info(h, i, C.byref(ql), C.byref(qb), C.byref(sd), C.byref(dt), C.byref(om)) == 0
        o = HybridChannel(ny, lay, kn, (-0.01, 0.01), n_half=nh, n_full=nf, qx=qx)
        nx = len(o.xx)
        assert (ql.value, qb.value) == (nx * 2 * nh, nx * nf)
        assert sd.value == 2 * lay * ql.value + (ny - 2 * lay) * qb.value == o.pack(o.equilibrium()).size
        assert dt.value == o.dt and om.value == o.omega
        total += (sd.value * 8 + 255) // 256 * 256
    assert L.lib.fdlb_hybrid_state_bytes(h) == total
    assert L.lib.fdlb_hybrid_step(h, 1) == L.ESTATE
    assert L.lib.fdlb_hybrid_info(h, 9, None, None, None, None, None) == L.EINVAL
    L.lib.fdlb_hybrid_destroy(h)
    bad = [dict(ny=1, layer=1), dict(ny=20, layer=0), dict(ny=20, layer=11), dict(kn=0.0), dict(n_half=1),
           dict(n_half=9), dict(n_full=1), dict(n_full=17), dict(qx=("full", 1)), dict(qx=("half", 1))]
    base = dict(ny=20, layer=4, kn=0.1, u_w=(-0.01, 0.01), n_half=2, n_full=2, qx=("full", 3))
    for b in bad:
        code, _ = _hybrid_create(F, [L.make_hybrid_desc(**dict(base, **b))])
        assert code == L.EINVAL, b
    for b in (dict(cfl=1.5), dict(kn=1e-4)):
        code, _ = _hybrid_create(F, [L.make_hybrid_desc(**dict(base, **b))])
        assert code == L.EUNSTABLE, b
    assert L.lib.fdlb_hybrid_create(None, 1, C.byref(C.c_void_p())) == L.EINVAL
