"""GPU parity of three-qubit gates (qf_instantiate3, qf_optimize_gate3): the
k = 3 case of the gate-set variants (Sec. III-A-3), against the FP64 oracle
whose k-qubit forms are pinned in test_oracle_pins.py.

Tolerances: complex128 sweeps follow the oracle's trajectory update by update
(gates to 1e-9 after a few sweeps, costs to 1e-10); complex64 builders to
1e-5 in the costs (1e-4 in the gates after three sweeps), with the 8 x 8
products on the matrix cores for n >= 8; the 8 x 8 update (Newton polar
iteration, Jacobi SVD for ill-conditioned environments) is unitary to 1e-12
and attains the nuclear norm to 1e-12 relative."""
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


NOPLATEAU = dict(diff_tol_r=0.0, long_diff_count=0)


def test_optimize_gate3_vs_oracle(qf):
    rng = np.random.default_rng(3100)
    envs = []
    for k in range(48):
        E = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
        if k % 8 == 1:
            E = 2.0 * I.haar_unitary(rng, 8)                       # scaled unitary
        if k % 8 == 2:
            E[:, 5] = 0.5 * E[:, 0] - 1j * E[:, 3]                # rank 7
        if k % 8 == 3:
            E[k % 8, :] = 0.0                                     # zero row
        if k % 8 == 4:
            E[[0, 6], :] = 0.0                                    # rank 6 by rows, plus a zero column
            E[:, 2] = 0.0
        if k % 8 == 5:
            E = 1e-200 * E                                        # tiny scale
        if k % 8 == 6:
            d = np.diag([1.0, 0.5, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
            E = I.haar_unitary(rng, 8) @ d @ I.haar_unitary(rng, 8)  # ill conditioned
        envs.append(E)
    E = np.stack(envs)
    U0 = np.stack([I.haar_unitary(rng, 8) for _ in range(48)])
    for beta in (0.0, 0.3):
        got = host(qf.optimize_gate3(dev(E), dev(U0), beta))
        M = (1 - beta) * E + beta * np.conj(np.swapaxes(U0, -1, -2))
        for k in range(48):
            assert np.abs(got[k].conj().T @ got[k] - np.eye(8)).max() < 1e-12, k
            sv = np.linalg.svd(M[k], compute_uv=False)
            kappa = sv[0] / sv[-1] if sv[-1] > 0 else np.inf
            if kappa < 1e10:
                ref = O.optimize_gate(E[k], U0[k], beta)
                assert np.abs(got[k] - ref).max() < max(1e-12, 1e-14 * kappa) * 10, k
            Mn = M[k] / np.abs(M[k]).max()
            svn = np.linalg.svd(Mn, compute_uv=False)
            assert abs(np.real(np.trace(Mn @ got[k])) - svn.sum()) <= 1e-12 * svn.sum(), k
    Z = np.zeros((2, 8, 8), complex)
    Z[1, 3, 3] = np.nan
    got = host(qf.optimize_gate3(dev(Z), dev(U0[:2]), 0.0))
    np.testing.assert_array_equal(got[0], U0[0])
    assert np.all(np.isnan(got[1]))


def test_optimize_gate3_condition_sweep(qf):
    """The 8 x 8 update for environments whose condition number sweeps 1 ..
    1e7 (|M|_F^2 |M^-1|_F^2 from 64 to beyond 1e14), across the point where
    the update hands over from the Newton polar iteration (< 1e8) to the
    Jacobi SVD: unitary to 1e-12, the polar factor to the condition-number
    bound of the LAPACK comparison, the attained value the nuclear norm, on
    both sides alike."""
    rng = np.random.default_rng(3300)
    envs = []
    for k in range(64):
        lo = -7.0 * k / 63.0  # smallest singular value 1 .. 1e-7
        s = np.sort(10.0 ** rng.uniform(lo, 0.0, 8))[::-1]
        s[0], s[-1] = 1.0, 10.0 ** lo
        E = I.haar_unitary(rng, 8) @ np.diag(s) @ I.haar_unitary(rng, 8)
        envs.append(E * 10.0 ** rng.uniform(-3, 3))
    E = np.stack(envs)
    U0 = np.stack([I.haar_unitary(rng, 8) for _ in range(64)])
    got = host(qf.optimize_gate3(dev(E), dev(U0), 0.0))
    c2 = []
    for k in range(64):
        ref = O.optimize_gate(E[k], U0[k], 0.0)
        assert np.abs(got[k].conj().T @ got[k] - np.eye(8)).max() < 1e-12, k
        sv = np.linalg.svd(E[k], compute_uv=False)
        kappa = sv[0] / sv[-1]
        c2.append(np.sum(sv ** 2) * np.sum(sv ** -2.0))
        assert np.abs(got[k] - ref).max() < max(1e-12, 1e-14 * kappa) * 10, (k, kappa)
        Mn = E[k] / np.abs(E[k]).max()
        svn = np.linalg.svd(Mn, compute_uv=False)
        assert abs(np.real(np.trace(Mn @ got[k])) - svn.sum()) <= 1e-12 * svn.sum(), k
    c2 = np.asarray(c2)
    assert (c2 < 1e7).sum() >= 10 and (c2 > 1e9).sum() >= 10  # both forms ran


@pytest.mark.parametrize("n,layers,S,sweeps", [(5, 4, 2, 3), (7, 4, 2, 2)])
def test_instantiate3_follows_oracle_c128(qf, n, layers, S, sweeps):
    """Fixed number of sweeps (plateau tests off), complex128: every start's
    gates and FP64 costs equal the oracle's builder-mode run."""
    pr = I.k3_problem(34, n, layers, S)
    rng = np.random.default_rng(3200 + n)
    V = I.haar_unitary(rng, 1 << n)
    res = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=sweeps, history_rows=sweeps + 1,
                          **NOPLATEAU)
    ref = O.instantiate(V, pr.init_gates, pr.locs, n, tol=1e-300, opt=O.Options(max_iter=sweeps, **NOPLATEAU))
    assert res.sweeps == ref.sweeps == sweeps
    assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-9
    assert np.abs(res.costs - ref.costs).max() <= 1e-10
    assert np.abs(res.history - ref.history[: res.history.shape[0]]).max() <= 1e-10


def test_instantiate3_n10_one_sweep_both_precisions(qf):
    """n = 10 three-qubit brick-wall (8 gates), two starts, one sweep: the
    complex128 gates match the oracle to 1e-9; complex64 ends within 1e-5
    of the oracle's costs (FP64 final costs of its own gates)."""
    n = 10
    pr = I.k3_problem(35, n, 3, 2)
    rng = np.random.default_rng(3300)
    V = I.haar_unitary(rng, 1 << n)
    ref = O.instantiate(V, pr.init_gates, pr.locs, n, tol=1e-300, opt=O.Options(max_iter=1, **NOPLATEAU))
    r128 = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=1, **NOPLATEAU)
    assert np.abs(host(r128.all_gates) - ref.all_gates).max() <= 1e-9
    assert np.abs(r128.costs - ref.costs).max() <= 1e-10
    r64 = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=1, precision=1, **NOPLATEAU)
    assert np.abs(r64.costs - ref.costs).max() <= 1e-5
    for s in range(2):
        assert abs(O.cost(V, host(r64.all_gates)[s], pr.locs, n) - r64.costs[s]) <= 1e-12


@pytest.mark.parametrize("n,layers,S,sweeps", [(8, 3, 2, 2), (9, 3, 2, 1)])
def test_instantiate3_c128_tiled_pass_follows_oracle(qf, n, layers, S, sweeps):
    """n >= 8: complex128 passes run on the two-gate pass's tiles (8 row
    variants x 8 column variants x 32 rest columns, address-order loads and
    stores); n = 8 is the smallest builder they fit.  Gates within 1e-9 and
    costs within 1e-10 of the oracle."""
    pr = I.k3_problem(40, n, layers, S)
    rng = np.random.default_rng(3600 + n)
    V = I.haar_unitary(rng, 1 << n)
    res = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=sweeps, history_rows=sweeps + 1,
                          **NOPLATEAU)
    ref = O.instantiate(V, pr.init_gates, pr.locs, n, tol=1e-300, opt=O.Options(max_iter=sweeps, **NOPLATEAU))
    assert res.sweeps == ref.sweeps == sweeps
    assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-9
    assert np.abs(res.costs - ref.costs).max() <= 1e-10
    assert np.abs(res.history - ref.history[: res.history.shape[0]]).max() <= 1e-10


@pytest.mark.parametrize("n", [8, 9])
def test_instantiate3_c64_matrix_core_pass_follows_oracle(qf, n):
    """n >= 8: the complex64 pass runs its 8 x 8 products on the matrix
    cores (n = 8: 32-group tiles of k_pass8_pipe; n >= 9: the two-gate
    pass's 64-column tiles).  Three sweeps from three Haar starts: the
    complex64 sweep costs stay within 1e-5 of the oracle's, the gates within
    1e-4, and the FP64 final costs equal the oracle cost of the returned
    gates."""
    pr = I.k3_problem(38, n, 3, 3)
    rng = np.random.default_rng(3400 + n)
    V = I.haar_unitary(rng, 1 << n)
    sweeps = 3
    ref = O.instantiate(V, pr.init_gates, pr.locs, n, tol=1e-300, opt=O.Options(max_iter=sweeps, **NOPLATEAU))
    r64 = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=sweeps, precision=1,
                          history_rows=sweeps + 1, **NOPLATEAU)
    assert r64.sweeps == ref.sweeps == sweeps
    assert np.abs(r64.history - ref.history[: r64.history.shape[0]]).max() <= 1e-5
    got = host(r64.all_gates)
    assert np.abs(got - ref.all_gates).max() <= 1e-4
    for s in range(3):
        assert abs(O.cost(V, got[s], pr.locs, n) - r64.costs[s]) <= 1e-12


def test_instantiate3_n10_eight_starts_pipelined_walk(qf):
    """n = 10, 8 starts: the launch configuration the three-qubit timing
    uses.  The pass then has 1024 (complex64) or 2048 (complex128) tiles per
    start set on half as many workgroups, so every workgroup walks two
    tiles and prefetches the second while it finishes the first.  One sweep: complex64
    costs within 1e-5 of the oracle's, gates within 1e-4, FP64 final costs
    equal to the oracle cost of the returned gates; complex128 gates within
    1e-9."""
    n = 10
    pr = I.k3_problem(39, n, 3, 8)
    rng = np.random.default_rng(3500)
    V = I.haar_unitary(rng, 1 << n)
    ref = O.instantiate(V, pr.init_gates, pr.locs, n, tol=1e-300, opt=O.Options(max_iter=1, **NOPLATEAU))
    r64 = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=1, precision=1, **NOPLATEAU)
    assert np.abs(r64.costs - ref.costs).max() <= 1e-5
    got = host(r64.all_gates)
    assert np.abs(got - ref.all_gates).max() <= 1e-4
    for s in (0, 7):
        assert abs(O.cost(V, got[s], pr.locs, n) - r64.costs[s]) <= 1e-12
    r128 = qf.instantiate3(dev(V), pr.locs, dev(pr.init_gates), tol=1e-300, max_iter=1, **NOPLATEAU)
    assert np.abs(host(r128.all_gates) - ref.all_gates).max() <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_instantiate3_converges_on_reachable_target(qf, precision):
    """A target built from three-qubit gates (n = 5, 3 gates), four Haar
    starts: the library converges like the oracle and the returned gates'
    FP64 oracle cost is below tol."""
    n = 5
    pr = I.k3_problem(36, n, 3, 4)
    tol = 1e-8
    res = qf.instantiate3(dev(pr.target), pr.locs, dev(pr.init_gates), tol=tol, precision=precision, max_iter=3000)
    ref = O.instantiate(pr.target, pr.init_gates, pr.locs, n, tol=tol, opt=O.Options(max_iter=3000))
    assert ref.status == O.STATUS_CONVERGED
    assert res.status == 0
    assert O.cost(pr.target, host(res.gates), pr.locs, n) < tol
    if precision == 0:
        # starts that all reach round-off tie, so the best start is not unique:
        # compare the sweep count and the best cost
        assert res.sweeps == ref.sweeps
        assert res.costs[res.best_start] <= ref.costs.min() + 1e-12


def test_instantiate3_rejects_invalid(qf):
    from paper_2306_08152_amd import QfError
    pr = I.k3_problem(37, 4, 2, 1)
    V = dev(pr.target)
    g = dev(pr.init_gates)
    with pytest.raises(QfError):
        qf.instantiate3(V, np.array([[0, 1, 1], [1, 2, 3]]), g)           # repeated qubit
    with pytest.raises(QfError):
        qf.instantiate3(V, np.array([[0, 1, 4], [1, 2, 3]]), g)           # qubit out of range
    with pytest.raises(QfError):
        qf.instantiate3(V, pr.locs, g, gate_kinds=[0, 0])                 # kinds are for 4 x 4 gates
    with pytest.raises(QfError):
        qf.instantiate3(V, pr.locs, g, mode=1)                            # streaming only
    with pytest.raises(QfError):
        qf.optimize_gate3(dev(np.zeros((1, 8, 8), complex)), dev(pr.init_gates[0, :1]), beta=2.0)


@pytest.mark.parametrize("precision", [1, 0])
def test_instantiate3_stream_groups_bitwise_equal(qf, precision):
    """The starts in 1 (the default), 2 or 3 staggered groups on separate
    streams: every start sees the same kernels in the same order, so gates
    and costs are bitwise the same (n = 10, 8 starts, one sweep)."""
    n = 10
    pr = I.k3_problem(39, n, 3, 8)
    V = dev(I.haar_unitary(np.random.default_rng(3500), 1 << n))
    g = dev(pr.init_gates)
    kw = dict(tol=1e-300, max_iter=1, precision=precision, **NOPLATEAU)
    a = qf.instantiate3(V, pr.locs, g, **kw)
    for groups in (1, 2, 3):
        b = qf.instantiate3(V, pr.locs, g, stream_groups=groups, **kw)
        assert np.array_equal(host(a.all_gates), host(b.all_gates)), groups
        assert np.array_equal(a.costs, b.costs), groups
