"""GPU parity: every step of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Tolerances: complex128 results agree with the oracle to 1e-10 (north-star
bar; entries here are O(1), rounding differences are ~1e-14); complex64
builder entries to 1e-5 relative to the largest entry; FP64 environments and
gate updates computed from the same complex64 values to 1e-12; final costs of
complex64 runs are FP64 re-evaluations and agree with the oracle's cost of the
returned gates to 1e-12."""
import numpy as np
import pytest

import oracle as O
import qfinputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def pairs(n):
    return [(a, b) for a in range(n) for b in range(n) if a != b]


C128_TOL = 1e-10
C64_REL = 1e-5


# --------------------------------------------------------------- apply / build

@pytest.mark.parametrize("n", [2, 3, 5, 8, 10, 11])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_gate_every_pair(qf, n, dtype):
    """Every ordered qubit pair exercises every tile geometry (local bits
    inside one segment, split into two segments, or four segments)."""
    rng = np.random.default_rng(1000 + n)
    S = 2
    X0 = I.random_builder(rng, S, n)
    if dtype == "c64":
        X0 = X0.astype(np.complex64).astype(np.complex128)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    prs = pairs(n)
    if n >= 10:
        prs = prs[::3] + [(0, 1), (1, 0), (n - 1, n - 2), (n - 2, n - 1), (0, n - 1), (n - 1, 0)]
    for k, loc in enumerate(prs):
        u = np.stack([I.haar_unitary(rng, 4) for _ in range(S)])
        side = k % 2
        dag = (k // 2) % 2
        X = dev(X0).to(tdt)
        qf.apply_gate(X, loc, dev(u), side, bool(dag))
        got = host(X).astype(np.complex128)
        uu = np.conj(np.swapaxes(u, -1, -2)) if dag else u
        ref = O.apply_left(X0, uu, loc, n) if side == 0 else O.apply_right(X0, uu, loc, n)
        scale = np.abs(ref).max()
        tol = C128_TOL * scale if dtype == "c128" else C64_REL * scale
        assert np.abs(got - ref).max() <= tol, (loc, side, dag)


@pytest.mark.parametrize("n,S", [(3, 1), (6, 3), (10, 2)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_build_matches_oracle_builder(qf, n, S, dtype):
    rng = np.random.default_rng(7 + n)
    p = 9
    locs = np.asarray([tuple(rng.choice(n, 2, replace=False)) for _ in range(p)], np.int32)
    V = I.haar_unitary(rng, 1 << n)
    gates = np.stack([I.haar_gates(rng, p) for _ in range(S)])
    X = qf.build(dev(V), locs, dev(gates), torch.complex128 if dtype == "c128" else torch.complex64)
    got = host(X).astype(np.complex128)
    ref = O.BuilderOracle(V, gates, locs, n).X
    tol = C128_TOL if dtype == "c128" else C64_REL * np.abs(ref).max()
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_build_n12_sampled_rows(qf, dtype):
    """Full-size builder (n = 12, 44 gates): rows sampled one by one by the
    oracle."""
    pr = I.config5(n_starts=1, build_target=False)
    rng = np.random.default_rng(12)
    V = I.haar_unitary(rng, 1 << 12)  # a generic unitary stands in for the target here
    X = qf.build(dev(V), pr.locs, dev(pr.init_gates), torch.complex128 if dtype == "c128" else torch.complex64)
    rows = [0, 1, 777, 2048, 4095]
    got = host(X[0, rows]).astype(np.complex128)
    ref = O.builder_rows(V, pr.init_gates[0], pr.locs, 12, rows)
    tol = C128_TOL if dtype == "c128" else C64_REL * np.abs(ref).max()
    assert np.abs(got - ref).max() <= tol


# --------------------------------------------------------------- environment

@pytest.mark.parametrize("n", [2, 4, 7, 10, 12])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_environment(qf, n, dtype):
    rng = np.random.default_rng(50 + n)
    S = 3 if n < 12 else 1
    X0 = I.random_builder(rng, S, n)
    if dtype == "c64":
        X0 = X0.astype(np.complex64).astype(np.complex128)
    X = dev(X0).to(torch.complex128 if dtype == "c128" else torch.complex64)
    prs = pairs(n) if n <= 4 else [(0, 1), (1, 0), (0, n - 1), (n - 1, 0), (n - 2, n - 1), (n // 2, 1)]
    for loc in prs:
        got = host(qf.environment(X, loc))
        ref = O.partial_trace(X0, loc, n)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), loc


def test_environment_alternating_layouts(qf):
    """Stand-alone calls with different (n, S) reuse the same context scratch;
    each must start from cleared arrival counters."""
    rng = np.random.default_rng(77)
    cases = [(12, 1), (10, 3), (11, 2), (10, 1), (12, 2), (9, 4)]
    for n, S in cases + cases[::-1]:
        X0 = I.random_builder(rng, S, n)
        got = host(qf.environment(dev(X0), (0, 1)))
        ref = O.partial_trace(X0, (0, 1), n)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), (n, S)


def test_standalone_calls_in_chunks(qf):
    """More builders than the stand-alone calls take per launch (they walk
    their builders in chunks of 1024 through the context's fixed scratch):
    every builder's environment and update equal the oracle's."""
    rng = np.random.default_rng(2400)
    n, S = 4, 2500
    X0 = I.random_builder(rng, S, n)
    loc = (1, 3)
    got = host(qf.environment(dev(X0), loc))
    ref = O.partial_trace(X0, loc, n)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    V = I.haar_unitary(rng, 1 << n)
    locs = np.array([loc, (0, 2)], np.int32)
    gates = np.stack([I.haar_gates(rng, 2) for _ in range(S)])
    ob = O.BuilderOracle(V, gates, locs, n)
    X = qf.build(dev(V), locs, dev(gates), torch.complex128)
    rec = []
    ob.update(1, 0, record=rec)
    gcol = dev(gates[:, 1].copy())
    _, env = qf.update_gate(X, tuple(locs[1]), 0, gcol, 0.0, want_env=True)
    assert np.abs(host(env) - rec[0][2]).max() <= 1e-10 * max(1.0, np.abs(rec[0][2]).max())
    assert np.abs(host(gcol) - rec[0][3]).max() <= 1e-9
    assert np.abs(host(X) - ob.X).max() <= C128_TOL


@pytest.mark.parametrize("n,S", [(11, 1), (12, 1), (12, 3), (13, 1)])
def test_environment_spread_over_workgroups(qf, n, S):
    """Few builders of n >= 11: the partial trace of each is spread over
    several workgroups (finished by the last to arrive); the sums equal the
    oracle's for every start, and a repeated call gives bitwise the same
    values (the hand-off sums the partials in workgroup order)."""
    rng = np.random.default_rng(1100 + 10 * n + S)
    X0 = (rng.standard_normal((S, 1 << n, 1 << n)) + 1j * rng.standard_normal((S, 1 << n, 1 << n)))
    X0 = X0.astype(np.complex64)
    X = dev(X0)
    for loc in [(0, 1), (n - 1, 2), (n // 2, n - 2)]:
        got = host(qf.environment(X, loc))
        ref = O.partial_trace(X0.astype(np.complex128), loc, n)
        assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max()), loc
        assert np.array_equal(got, host(qf.environment(X, loc)))
    del X
    torch.cuda.empty_cache()


# --------------------------------------------------------------- gate update

def test_optimize_gate_vs_lapack(qf):
    rng = np.random.default_rng(99)
    envs = []
    for k in range(64):
        E = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        if k % 8 == 1:
            E = 3.0 * I.haar_unitary(rng, 4)                   # scaled unitary
        if k % 8 == 2:
            E[:, 2] = 0.3 * E[:, 0] - 1j * E[:, 1]              # rank 3
        if k % 8 == 3:
            d = np.diag([1.0, 1e-3, 1e-6, 1e-9])
            E = I.haar_unitary(rng, 4) @ d @ I.haar_unitary(rng, 4)  # ill conditioned
        if k % 8 == 4:
            E = 1e-200 * E                                       # tiny scale
        if k % 8 == 5:
            E[k % 4, :] = 0.0                                    # zero row: rank 3 that no column shows
        if k % 8 == 6:
            E[[0, 3], :] = 0.0                                   # two zero rows and a zero column
            E[:, 1] = 0.0
        envs.append(E)
    E = np.stack(envs)
    U0 = np.stack([I.haar_unitary(rng, 4) for _ in range(64)])
    for beta in (0.0, 0.25):
        got = host(qf.optimize_gate(dev(E), dev(U0), beta))
        M = (1 - beta) * E + beta * np.conj(np.swapaxes(U0, -1, -2))
        for k in range(64):
            ref = O.optimize_gate(E[k], U0[k], beta)
            assert np.abs(got[k].conj().T @ got[k] - np.eye(4)).max() < 1e-12
            sv = np.linalg.svd(M[k], compute_uv=False)
            kappa = sv[0] / sv[-1] if sv[-1] > 0 else np.inf
            if kappa < 1e10:
                # unique polar factor, determined to about eps * condition number
                assert np.abs(got[k] - ref).max() < max(1e-12, 1e-14 * kappa) * 10, k
            # the attained value is the nuclear norm in every case (checked on
            # M / max|M| so that tiny environments do not underflow)
            Mn = M[k] / np.abs(M[k]).max()
            svn = np.linalg.svd(Mn, compute_uv=False)
            val = np.real(np.trace(Mn @ got[k]))
            assert abs(val - svn.sum()) <= 1e-12 * svn.sum(), k
    # zero environment keeps the gate; NaN gives NaN
    Z = np.zeros((2, 4, 4), complex)
    Z[1, 0, 0] = np.nan
    got = host(qf.optimize_gate(dev(Z), dev(U0[:2]), 0.0))
    np.testing.assert_array_equal(got[0], U0[0])
    assert np.all(np.isnan(got[1]))


def test_optimize_gate_condition_sweep(qf):
    """The update for environments whose condition number sweeps 1 .. 1e7
    (squared Frobenius condition number |M|_F^2 |M^-1|_F^2 from about 16 to
    1e15), across the point where the hex form hands over from the Newton
    polar iteration (|M|_F^2 |M^-1|_F^2 < 1e6) to the Jacobi SVD: unitary to
    1e-12, the polar factor to the condition-number bound of the LAPACK
    comparison, the attained value the nuclear norm, on both sides alike."""
    rng = np.random.default_rng(7)
    envs = []
    for k in range(96):
        lo = -7.0 * k / 95.0  # smallest singular value 1 .. 1e-7
        s = np.sort(10.0 ** rng.uniform(lo, 0.0, 4))[::-1]
        s[0], s[-1] = 1.0, 10.0 ** lo
        E = I.haar_unitary(rng, 4) @ np.diag(s) @ I.haar_unitary(rng, 4)
        envs.append(E * 10.0 ** rng.uniform(-3, 3))
    E = np.stack(envs)
    U0 = np.stack([I.haar_unitary(rng, 4) for _ in range(96)])
    got = host(qf.optimize_gate(dev(E), dev(U0), 0.0))
    c2 = []
    for k in range(96):
        ref = O.optimize_gate(E[k], U0[k], 0.0)
        assert np.abs(got[k].conj().T @ got[k] - np.eye(4)).max() < 1e-12, k
        sv = np.linalg.svd(E[k], compute_uv=False)
        kappa = sv[0] / sv[-1]
        c2.append(np.sum(sv ** 2) * np.sum(sv ** -2.0))
        assert np.abs(got[k] - ref).max() < max(1e-12, 1e-14 * kappa) * 10, (k, kappa)
        Mn = E[k] / np.abs(E[k]).max()
        svn = np.linalg.svd(Mn, compute_uv=False)
        assert abs(np.real(np.trace(Mn @ got[k])) - svn.sum()) <= 1e-12 * svn.sum(), k
    c2 = np.asarray(c2)
    assert (c2 < 1e5).sum() >= 10 and (c2 > 1e7).sum() >= 10  # both forms ran


@pytest.mark.parametrize("n", [3, 7, 10])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_update_gate_steps(qf, n, dtype):
    """A run of single TwoSidedSweep updates through qf_update_gate against
    the oracle's builder mode, update by update."""
    rng = np.random.default_rng(300 + n)
    S, p = 2, 6
    locs = np.asarray([tuple(rng.choice(n, 2, replace=False)) for _ in range(p)], np.int32)
    V = I.haar_unitary(rng, 1 << n)
    gates = np.stack([I.haar_gates(rng, p) for _ in range(S)])
    ob = O.BuilderOracle(V, gates, locs, n)
    X = qf.build(dev(V), locs, dev(gates), torch.complex128 if dtype == "c128" else torch.complex64)
    G = dev(gates.copy())
    steps = [(g, 0) for g in range(p - 1, -1, -1)] + [(g, 1) for g in range(p)]
    for g, half in steps:
        rec = []
        Xb = X.to(torch.complex128) if dtype == "c64" else None
        if dtype == "c64":
            # the oracle starts each step from the GPU's complex64 builder
            ob.X = host(Xb)
            ob.gates = host(G).copy()
        ob.update(g, half, record=rec)
        gcol = G[:, g].contiguous()
        _, env = qf.update_gate(X, tuple(locs[g]), half, gcol, 0.0, want_env=True)
        G[:, g] = gcol
        E_ref, u_ref = rec[0][2], rec[0][3]
        assert np.abs(host(env) - E_ref).max() <= 1e-10 * max(1.0, np.abs(E_ref).max()), (g, half)
        assert np.abs(host(gcol) - u_ref).max() <= 1e-9, (g, half)
        tol = C128_TOL if dtype == "c128" else C64_REL * np.abs(ob.X).max()
        assert np.abs(host(X).astype(np.complex128) - ob.X).max() <= tol, (g, half)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pass_forms_bitwise_equal(qf, dtype):
    """Every form of the fused pass (register-direct, micro-tile for
    complex64, LDS tiles of every width) gives bitwise the same builder for
    one-sided products of both sides and for the two-sided update, at every
    qubit pair of n = 6 and a spread of pairs (all six ordered pairs of the
    three lowest bits included) of n = 9 and 10; the one-sided products also
    match the oracle."""
    prec = 0 if dtype == "c128" else 1
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    forms = [-1, 256, 512] + ([1024, -2] if dtype == "c64" else [])
    S = 2
    try:
        for n in (6, 7, 9, 10):
            rng = np.random.default_rng(4000 + n)
            X0 = I.random_builder(rng, S, n)
            if dtype == "c64":
                X0 = X0.astype(np.complex64).astype(np.complex128)
            prs = pairs(n)
            if n == 9:
                prs = prs[::9] + [(7, 8), (8, 7), (6, 7), (7, 6), (6, 8), (8, 6)]
            if n == 10:
                prs = prs[::5] + [(8, 9), (9, 8), (7, 8), (8, 7), (7, 9), (9, 7), (0, 9), (9, 0)]
            for k, loc in enumerate(prs):
                u = np.stack([I.haar_unitary(rng, 4) for _ in range(S)])
                w = np.stack([I.haar_unitary(rng, 4) for _ in range(S)])
                gq = np.stack([I.haar_unitary(rng, 4) for _ in range(S)])
                outs = []
                for f in forms:
                    for cls in (0, 1):
                        qf.set_pass_tile("cuda", prec, n, cls, f)
                    X = dev(X0).to(tdt)
                    qf.apply_gate(X, loc, dev(u), 0, False)
                    qf.apply_gate(X, loc, dev(w), 1, True)
                    one = host(X).astype(np.complex128)
                    G = dev(gq.copy())
                    qf.update_gate(X, loc, k % 2, G)
                    outs.append((one, host(X), host(G)))
                ref = O.apply_right(O.apply_left(X0, u, loc, n), np.conj(np.swapaxes(w, -1, -2)), loc, n)
                tol = C128_TOL if dtype == "c128" else C64_REL * np.abs(ref).max()
                assert np.abs(outs[0][0] - ref).max() <= tol, (n, loc)
                for f, o in zip(forms[1:], outs[1:]):
                    assert np.array_equal(o[0], outs[0][0]), (n, loc, f)
                    assert np.array_equal(o[1], outs[0][1]), (n, loc, f)
                    assert np.array_equal(o[2], outs[0][2]), (n, loc, f)
    finally:
        for n in (6, 7, 10):
            for cls in (0, 1):
                qf.set_pass_tile("cuda", prec, n, cls, 0)


def test_cost_kernel(qf):
    rng = np.random.default_rng(5)
    X0 = I.random_builder(rng, 4, 9)
    c, tr = qf.cost(dev(X0))
    ref_tr = np.trace(X0, axis1=1, axis2=2)
    assert np.abs(host(tr) - ref_tr).max() < 1e-12
    assert np.abs(host(c) - (1 - np.abs(ref_tr) / 512)).max() < 1e-14


# --------------------------------------------------------------- instantiation

def _oracle_opts(**kw):
    return O.Options(**kw)


def _run_both(qf, pr, tol, mode, precision, max_iter=100000, plateau=True, starts=None, hist_rows=2000):
    init = pr.init_gates if starts is None else pr.init_gates[:starts]
    kw = {} if plateau else dict(diff_tol_r=0.0, long_diff_count=0)
    res = qf.instantiate(dev(pr.target), pr.locs, dev(init), tol=tol, mode=mode, precision=precision,
                         max_iter=max_iter, history_rows=hist_rows, **kw)
    ref = O.instantiate(pr.target, init, pr.locs, pr.n, tol=tol, opt=_oracle_opts(max_iter=max_iter, **kw))
    return res, ref


@pytest.mark.parametrize("mode", [1, 2])
def test_config1_c128(qf, mode):
    """n = 3, four U(4) gates, one start, c128, stop at 1e-10 or 1000 sweeps."""
    pr = I.config1()
    res, ref = _run_both(qf, pr, 1e-10, mode, 0, max_iter=1000, plateau=False, hist_rows=1001)
    assert res.sweeps == ref.sweeps and res.status == ref.status
    assert np.abs(res.history - ref.history[: res.history.shape[0]]).max() <= C128_TOL
    assert abs(res.costs[0] - ref.costs[0]) <= C128_TOL
    assert np.abs(host(res.gates) - ref.gates).max() <= 1e-8


@pytest.mark.parametrize("mode", [1, 2])
def test_config1_converging_start(qf, mode):
    pr = I.config1()
    pr.init_gates = I.haar_gates(I.rng_for(1, 1, 1000), 4)[None]
    res, ref = _run_both(qf, pr, 1e-10, mode, 0, max_iter=1000, plateau=False)
    assert ref.status == O.STATUS_CONVERGED
    assert res.status == 0 and res.sweeps == ref.sweeps
    assert res.costs[0] < 1e-10
    assert np.abs(res.history - ref.history[: res.history.shape[0]]).max() <= C128_TOL


@pytest.mark.parametrize("mode", [1, 2])
def test_config2_c128(qf, mode):
    """n = 6 brick-wall, 15 gates, 32 starts, tol 1e-8, default plateau tests."""
    pr = I.config2()
    res, ref = _run_both(qf, pr, 1e-8, mode, 0)
    assert res.sweeps == ref.sweeps and res.status == ref.status and res.best_start == ref.best_start
    assert np.abs(res.history - ref.history[: res.history.shape[0]]).max() <= C128_TOL
    assert np.abs(res.costs - ref.costs).max() <= C128_TOL
    assert res.costs[res.best_start] < 1e-8


@pytest.mark.parametrize("mode", [1, 2])
def test_config2_c64(qf, mode):
    """Complex64 builder with FP64 gate updates, tests and final cost: the
    returned costs are FP64 and equal the oracle's cost of the returned gates;
    the best start reaches the tolerance."""
    pr = I.config2()
    res = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-8, mode=mode, precision=1,
                         history_rows=2000)
    allg = host(res.all_gates)
    for s in range(pr.n_starts):
        c = O.cost(pr.target, allg[s], pr.locs, pr.n)
        assert abs(c - res.costs[s]) <= 1e-12, s
        assert np.abs(np.conj(np.swapaxes(allg[s], -1, -2)) @ allg[s] - np.eye(4)).max() < 1e-12
    assert res.status == 0 and res.costs[res.best_start] < 1e-8
    # the first sweep tracks the FP64 trajectory to complex64 accuracy
    ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-8, opt=O.Options(max_iter=1))
    assert np.abs(res.history[1] - ref.history[1]).max() <= 1e-5


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("cfg,n_starts", [(45, 3), (49, 4)])
def test_staggered_plateaus_match_oracle(qf, mode, cfg, n_starts):
    """Starts on an unreachable target whose plateau tests fire at different
    sweeps (config 45: 35, 7, 13; config 49: 13, 10, 12, 22, one of whose
    tests fires and later stops firing): the job runs until every start has
    hit a plateau, plateaued starts keep sweeping, and sweeps, status, best
    start, the whole cost history and the final costs equal the oracle's."""
    n, locs, V, init = I.unreachable_problem(cfg, n_starts)
    res = qf.instantiate(dev(V), locs, dev(init), tol=1e-10, mode=mode, precision=0, history_rows=200)
    ref = O.instantiate(V, init, locs, n, tol=1e-10)
    assert ref.status == O.STATUS_PLATEAU
    assert res.sweeps == ref.sweeps and res.status == ref.status and res.best_start == ref.best_start
    assert np.abs(res.history - ref.history).max() <= C128_TOL
    assert np.abs(res.costs - ref.costs).max() <= C128_TOL
    assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
def test_n10_streaming_two_sweeps(qf, precision):
    """Full-size n = 10 brick-wall (45 gates), two starts, two sweeps."""
    pr = I.config3(n_starts=2)
    res, ref = _run_both(qf, pr, 1e-8, 2, precision, max_iter=2, plateau=False)
    assert res.sweeps == 2 and ref.sweeps == 2
    tol = C128_TOL if precision == 0 else 1e-5
    assert np.abs(res.history - ref.history).max() <= tol
    assert np.abs(res.costs - ref.costs).max() <= (C128_TOL if precision == 0 else 1e-5)
    if precision == 0:
        assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-8


def test_n12_one_sweep_properties(qf):
    """n = 12 (44 gates), complex64, one sweep: the returned gates are
    unitary, the cost does not increase, and the FP64 cost of the returned
    gates matches a complex128 rebuild's trace."""
    pr = I.config5(n_starts=1, build_target=False)
    rng = np.random.default_rng(120)
    # target: a random circuit on the same structure (built on the CPU)
    tg = I.haar_gates(rng, pr.n_gates)
    V = I.circuit_unitary(tg, pr.locs, 12)
    res = qf.instantiate(dev(V), pr.locs, dev(pr.init_gates), tol=1e-8, mode=2, precision=1, max_iter=1,
                         diff_tol_r=0.0, long_diff_count=0, history_rows=2)
    g = host(res.all_gates)[0]
    assert np.abs(np.conj(np.swapaxes(g, -1, -2)) @ g - np.eye(4)).max() < 1e-12
    assert res.history[1, 0] <= res.history[0, 0] + 1e-6
    X = qf.build(dev(V), pr.locs, dev(g[None]), torch.complex128)
    c, _ = qf.cost(X)
    assert abs(host(c)[0] - res.costs[0]) < 1e-12
    # sampled rows of the complex128 rebuild against the oracle
    rows = [5, 3000]
    ref = O.builder_rows(V, g, pr.locs, 12, rows)
    assert np.abs(host(X[0, rows]) - ref).max() < C128_TOL


def _golden(name):
    import os
    return np.load(os.path.join(os.path.dirname(__file__), "golden", name), allow_pickle=False)


def test_n12_sweep_matches_oracle_update_by_update(qf):
    """Full-size n = 12 brick-wall (44 gates, 4096 x 4096 builder), complex128:
    every one of the 88 updates of the first TwoSidedSweep (environment, new
    gate, trace of the circuit tensor) against the oracle's builder mode
    (values stored by tests/golden/make_sweep_trajectories.py)."""
    gd = _golden("n12_brickwall8_sweep1.npz")
    pr = I.config5(n_starts=1)
    N = 1 << pr.n
    X = qf.build(dev(pr.target), pr.locs, dev(pr.init_gates), torch.complex128)
    c0, _ = qf.cost(X)
    assert abs(host(c0)[0] - float(gd["cost0"])) <= C128_TOL
    G = dev(pr.init_gates.copy())
    for j, (g, half) in enumerate(gd["order"]):
        gcol = G[:, g].contiguous()
        _, env = qf.update_gate(X, tuple(pr.locs[g]), int(half), gcol, 0.0, want_env=True)
        G[:, g] = gcol
        E_ref = gd["env"][j]
        assert np.abs(host(env)[0] - E_ref).max() <= C128_TOL * max(1.0, np.abs(E_ref).max()), (j, g, half)
        assert np.abs(host(gcol)[0] - gd["gate"][j]).max() <= 1e-9, (j, g, half)
        _, tr = qf.cost(X)
        assert abs(host(tr)[0] - gd["trace"][j]) <= C128_TOL * N, (j, g, half)
    assert np.abs(host(G)[0] - gd["gates1"]).max() <= 1e-9
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [0, 1])
def test_n12_instantiate_one_sweep_matches_oracle(qf, precision):
    """qf_instantiate on the n = 12 workload for one sweep (streaming, one
    start): complex128 cost history, FP64 final cost and gates to the
    complex128 bar; complex64 cost after the sweep to 1e-5, its final cost an
    FP64 re-evaluation of its own gates (unitary to 1e-12)."""
    gd = _golden("n12_brickwall8_sweep1.npz")
    pr = I.config5(n_starts=1)
    res = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-8, mode=2, precision=precision,
                         max_iter=1, diff_tol_r=0.0, long_diff_count=0, history_rows=2)
    hist_ref = np.array([float(gd["cost0"]), float(gd["cost1"])])
    g = host(res.all_gates)[0]
    assert np.abs(np.conj(np.swapaxes(g, -1, -2)) @ g - np.eye(4)).max() < 1e-12
    if precision == 0:
        assert np.abs(res.history[:, 0] - hist_ref).max() <= C128_TOL
        assert abs(res.costs[0] - float(gd["cost1"])) <= C128_TOL
        assert np.abs(g - gd["gates1"]).max() <= 1e-9
    else:
        assert np.abs(res.history[:, 0] - hist_ref).max() <= C64_REL
        assert abs(res.costs[0] - float(gd["cost1"])) <= C64_REL
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [0, 1])
def test_n10_s16_default_schedule_matches_oracle(qf, precision):
    """The headline launch configuration (n = 10, 45 gates, 16 starts, the
    default streaming schedule with environment steps fused beside other
    groups' passes on two streams) for one sweep: starts 0, 7 and 15 against
    the oracle (values stored by tests/golden/make_sweep_trajectories.py)."""
    gd = _golden("n10_brickwall10_s16_sweep1.npz")
    pr = I.config3(n_starts=16)
    res = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-300, precision=precision,
                         max_iter=1, diff_tol_r=0.0, long_diff_count=0, history_rows=2)
    st = list(gd["starts"])
    tol = C128_TOL if precision == 0 else C64_REL
    assert np.abs(res.history[:, st] - gd["history"]).max() <= tol
    assert np.abs(res.costs[st] - gd["costs"]).max() <= tol
    if precision == 0:
        assert np.abs(host(res.all_gates)[st] - gd["gates"]).max() <= 1e-8


@pytest.mark.parametrize("S", [1, 3, 16])
def test_stream_schedules_bitwise_equal(qf, S):
    """The default schedule (group pairs, each launch one group's environment
    step beside another group's pass) and 1, 2 and 4 staggered groups on
    separate streams give bitwise the same gates and costs: every start sees
    the same kernels in the same order (n = 10, complex64, two sweeps)."""
    pr = I.config3(n_starts=S)
    kw = dict(tol=1e-300, max_iter=2, precision=1, diff_tol_r=0.0, long_diff_count=0)
    V, g = dev(pr.target), dev(pr.init_gates)
    a = qf.instantiate(V, pr.locs, g, **kw)
    for groups in (1, 2, 4):
        b = qf.instantiate(V, pr.locs, g, stream_groups=groups, **kw)
        assert np.array_equal(host(a.all_gates), host(b.all_gates)), groups
        assert np.array_equal(a.costs, b.costs), groups


def test_timing_run_same_results_and_consistent_durations(qf):
    """One pass per gate update (gate_pairs = 0): the per-kernel timing run
    (starts as one group, every pass and
    environment launch stamped by its own dispatch) gives bitwise the
    default schedule's gates and costs, counts 2p passes and 2p environment
    steps per sweep, and its kernels, which run one after another on one
    stream, sum to no more than the sweep loop's device time."""
    pr = I.config3(n_starts=4)
    sweeps = 2
    kw = dict(tol=1e-300, max_iter=sweeps, precision=1, diff_tol_r=0.0, long_diff_count=0, gate_pairs=0)
    V, g = dev(pr.target), dev(pr.init_gates)
    a = qf.instantiate(V, pr.locs, g, **kw)
    b = qf.instantiate(V, pr.locs, g, timing=True, **kw)
    assert np.array_equal(host(a.all_gates), host(b.all_gates))
    assert np.array_equal(a.costs, b.costs)
    t = b.timing
    p = len(pr.locs)
    assert t["pass_launches"] == 2 * p * sweeps
    assert t["env_launches"] == 2 * p * sweeps
    per_pass_us = 1e3 * t["pass_ms"] / t["pass_launches"]
    assert 1.0 < per_pass_us < 1e4
    assert 0 < t["env_ms"] and t["pass_ms"] + t["env_ms"] <= t["sweep_ms"] * 1.001


def test_stream_schedules_with_fixed_gates(qf):
    """U3 + CNOT at n = 9 (fixed CNOT steps have no environment, so the
    default schedule launches some passes alone): bitwise equal to one group."""
    locs, kinds, _, V, init = I.u3cx_problem(9, 9, 3, 6)
    kw = dict(tol=1e-300, max_iter=2, precision=1, diff_tol_r=0.0, long_diff_count=0, gate_kinds=kinds)
    a = qf.instantiate(dev(V), locs, dev(init), **kw)
    b = qf.instantiate(dev(V), locs, dev(init), stream_groups=1, **kw)
    assert np.array_equal(host(a.all_gates), host(b.all_gates))
    assert np.array_equal(a.costs, b.costs)


def test_determinism(qf):
    pr = I.config2(n_starts=8)
    a = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-8, max_iter=30)
    b = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-8, max_iter=30)
    assert np.array_equal(host(a.all_gates), host(b.all_gates))
    pr3 = I.config3(n_starts=1)
    a = qf.instantiate(dev(pr3.target), pr3.locs, dev(pr3.init_gates), tol=1e-8, max_iter=1, precision=1)
    b = qf.instantiate(dev(pr3.target), pr3.locs, dev(pr3.init_gates), tol=1e-8, max_iter=1, precision=1)
    assert np.array_equal(host(a.all_gates), host(b.all_gates))


def test_nan_start_frozen(qf):
    pr = I.config1()
    bad = pr.init_gates[0].copy()
    bad[2, 1, 1] = np.nan
    init = np.stack([bad, pr.target_gates])
    for mode in (1, 2):
        res = qf.instantiate(dev(pr.target), pr.locs, dev(init), tol=1e-10, mode=mode, max_iter=5)
        assert res.best_start == 1 and res.status == 0 and not np.isfinite(res.costs[0])


def test_invalid_arguments_rejected(qf):
    from paper_2306_08152_amd import QfError
    pr = I.config1()
    with pytest.raises(QfError):
        qf.instantiate(dev(pr.target), [(0, 0)] * 4, dev(pr.init_gates), tol=1e-8)
    with pytest.raises(QfError):
        qf.instantiate(dev(pr.target), [(0, 3)] * 4, dev(pr.init_gates), tol=1e-8)
    with pytest.raises(QfError):
        qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=-1.0)
    with pytest.raises(QfError):
        qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-8, mode=1, beta=2.0)


def test_environment_n15_multi_workgroup(qf):
    """n = 15 (environment summed by several workgroups per start): a sparse
    complex64 builder (random diagonal plus entries that couple the gate's
    local indices) whose partial trace is known entry by entry."""
    n, N = 15, 1 << 15
    rng = np.random.default_rng(1515)
    loc = (2, 11)
    b0, b1 = n - 1 - loc[0], n - 1 - loc[1]
    X = torch.zeros((1, N, N), dtype=torch.complex64, device="cuda")
    d = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    X[0].diagonal().copy_(torch.from_numpy(d).to("cuda"))
    ref = np.zeros((4, 4), np.complex128)
    idx = np.arange(N)
    li = (((idx >> b0) & 1) << 1) | ((idx >> b1) & 1)
    for i in range(4):
        ref[i, i] += d[li == i].astype(np.complex128).sum()
    # off-diagonal couplings: rows and columns that differ only in the gate bits
    for _ in range(64):
        rest = int(rng.integers(0, N)) & ~((1 << b0) | (1 << b1))
        i, j = rng.integers(0, 4, size=2)
        if i == j:
            continue
        r = rest | (int(i >> 1) << b0) | (int(i & 1) << b1)
        c = rest | (int(j >> 1) << b0) | (int(j & 1) << b1)
        v = np.complex64(rng.standard_normal() + 1j * rng.standard_normal())
        X[0, r, c] += torch.tensor(v, device="cuda")
        ref[i, j] += complex(v)
    got = host(qf.environment(X, loc))[0]
    assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    del X
    torch.cuda.empty_cache()
