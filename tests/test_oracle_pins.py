"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-types the oracle's own formula: each checks it against an
independent construction (dense Kronecker products, brute-force derivatives,
closed-form solutions, inequalities, invariants stated in the paper)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import qfinputs as I

RNG = np.random.default_rng(20230613)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def haar(d, rng=RNG):
    return I.haar_unitary(rng, d)


def rand_gates(p, rng=RNG):
    return np.stack([haar(4, rng) for _ in range(p)])


def rand_locs(n, p, rng=RNG):
    out = []
    for _ in range(p):
        a, b = rng.choice(n, size=2, replace=False)
        out.append((int(a), int(b)))
    return np.asarray(out, np.int32)


def all_pairs(n):
    return [(a, b) for a in range(n) for b in range(n) if a != b]


# ---------------------------------------------------------------- embedding

@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_embed_adjacent_is_textbook_kron(n):
    """Adjacent ascending pair (q, q+1): I_{2^q} (x) u (x) I_{2^(n-q-2)}."""
    u = haar(4)
    for q in range(n - 1):
        ref = np.kron(np.kron(np.eye(1 << q), u), np.eye(1 << (n - q - 2)))
        assert np.array_equal(O.embed(u, (q, q + 1), n), ref)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_embed_general_pairs_match_swap_network(n):
    u = haar(4)
    for loc in all_pairs(n):
        np.testing.assert_allclose(O.embed(u, loc, n), O.embed_kron(u, loc, n), atol=1e-15)


def test_embed_reversed_pair_is_swap_conjugate():
    """Gate on (1, 0) equals SWAP u SWAP on (0, 1)."""
    u = haar(4)
    sw = np.eye(4)[[0, 2, 1, 3]]
    np.testing.assert_allclose(O.embed(u, (1, 0), 2), sw @ u @ sw, atol=0)
    np.testing.assert_allclose(O.embed(u, (2, 0), 3), O.embed(sw @ u @ sw, (0, 2), 3), atol=1e-15)


@pytest.mark.parametrize("n", [3, 5])
def test_structured_apply_equals_dense(n):
    N = 1 << n
    X = I.random_builder(RNG, 1, n)[0]
    for loc in all_pairs(n)[:12]:
        u = haar(4)
        G = O.embed(u, loc, n)
        np.testing.assert_allclose(O.apply_left(X, u, loc, n), G @ X, atol=1e-13)
        np.testing.assert_allclose(O.apply_right(X, u, loc, n), X @ G, atol=1e-13)
    # batched, one gate per batch entry
    Xs = I.random_builder(RNG, 3, n)
    us = rand_gates(3)
    loc = (n - 1, 0)
    out = O.apply_left(Xs, us, loc, n)
    for s in range(3):
        np.testing.assert_allclose(out[s], O.embed(us[s], loc, n) @ Xs[s], atol=1e-13)
    out = O.apply_right(Xs, us, loc, n)
    for s in range(3):
        np.testing.assert_allclose(out[s], Xs[s] @ O.embed(us[s], loc, n), atol=1e-13)
    assert N == Xs.shape[-1]


def test_circuit_unitary_dense_structured_and_inputs_agree():
    n, p = 4, 7
    g = rand_gates(p)
    locs = rand_locs(n, p)
    Cd = O.circuit_unitary(g, locs, n, dense=True)
    Cs = O.circuit_unitary(g, locs, n)
    Ci = I.circuit_unitary(g, locs, n)
    np.testing.assert_allclose(Cs, Cd, atol=1e-13)
    np.testing.assert_allclose(Ci, Cd, atol=1e-13)
    np.testing.assert_allclose(Cd.conj().T @ Cd, np.eye(1 << n), atol=1e-13)
    # time order: C = G_p ... G_1
    ref = np.eye(1 << n)
    for u, l in zip(g, locs):
        ref = O.embed_kron(u, l, n) @ ref
    np.testing.assert_allclose(Cd, ref, atol=1e-13)


# ---------------------------------------------------------------- cost

def test_cost_closed_forms():
    n = 3
    V = haar(8)
    assert abs(1.0 - abs(O.overlap(V, V)) / 8) < 1e-15
    assert abs(1.0 - abs(O.overlap(V, np.exp(0.7j) * V)) / 8) < 1e-15  # global phase
    X = np.array([[0, 1], [1, 0]])
    C = np.kron(X, np.eye(4))                                          # traceless vs I
    assert abs(1.0 - abs(O.overlap(np.eye(8), C)) / 8 - 1.0) < 1e-15


def test_frobenius_identity_eq_cost():
    """||U - V||^2 = 2^(n+1) (1 - Re Tr(V^dagger U) / 2^n) (Eq. cost)."""
    for n in (2, 3, 5):
        N = 1 << n
        U, V = haar(N), haar(N)
        lhs = O.frobenius_distance_sq(V, U)
        rhs = 2 * N * (1 - np.real(O.overlap(V, U)) / N)
        assert abs(lhs - rhs) < 1e-12 * N


# ---------------------------------------------------------------- environment

@pytest.mark.parametrize("n", [2, 3, 4])
def test_partial_trace_forms_and_identity(n):
    X = I.random_builder(RNG, 1, n)[0]
    for loc in all_pairs(n):
        E = O.partial_trace(X, loc, n)
        np.testing.assert_allclose(E, O.partial_trace_loops(X, loc, n), atol=1e-14)
        u = RNG.standard_normal((4, 4)) + 1j * RNG.standard_normal((4, 4))
        # Tr((u (x) I) X) = Tr(E u) for any u (defines the orientation of E)
        lhs = np.trace(O.embed(u, loc, n) @ X)
        assert abs(lhs - np.trace(E @ u)) < 1e-13


def _problem(n, p, rng=RNG):
    locs = rand_locs(n, p, rng)
    V = haar(1 << n, rng)
    gates = rand_gates(p, rng)
    return V, gates, locs


@pytest.mark.parametrize("n,p", [(2, 3), (3, 5), (4, 6), (5, 8)])
def test_trace_invariant_every_gate(n, p):
    """Tr(E_g u_g) = Tr(V^dagger C) for every gate g (Sec. III)."""
    V, gates, locs = _problem(n, p)
    T = O.overlap(V, O.circuit_unitary(gates, locs, n, dense=True))
    for g in range(p):
        E = O.environment(V, gates, locs, n, g)
        assert abs(np.trace(E @ gates[g]) - T) < 1e-12 * (1 << n)


@pytest.mark.parametrize("n,p", [(2, 2), (3, 4), (4, 5)])
def test_environment_is_brute_force_derivative(n, p):
    """T is linear in u_g, so E_g[i, j] = T(u_g := e_{ji}) exactly, and a
    central difference of any step reproduces it (dense circuit products)."""
    V, gates, locs = _problem(n, p)

    def T_with(g, m):
        gg = [x for x in gates]
        gg[g] = m
        C = np.eye(1 << n, dtype=complex)
        for u, l in zip(gg, locs):
            C = O.embed(u, l, n) @ C
        return np.trace(V.conj().T @ C)

    for g in range(p):
        E = O.environment(V, gates, locs, n, g)
        brute = np.zeros((4, 4), complex)
        for i in range(4):
            for j in range(4):
                unit = np.zeros((4, 4), complex)
                unit[j, i] = 1.0
                brute[i, j] = T_with(g, unit)
        np.testing.assert_allclose(E, brute, atol=1e-13)
        # central difference around the current gate, h = 1e-4
        i, j = 1, 2
        unit = np.zeros((4, 4), complex)
        unit[j, i] = 1.0
        fd = (T_with(g, gates[g] + 1e-4 * unit) - T_with(g, gates[g] - 1e-4 * unit)) / 2e-4
        assert abs(fd - E[i, j]) < 1e-9


# ---------------------------------------------------------------- gate update

def test_update_unitary_and_locally_optimal():
    """u_new is unitary and maximises Re Tr(E u) over unitaries: the value is
    the nuclear norm of E and no Haar unitary does better (Sec. III-A-1)."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        E = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        if trial == 0:
            E[:, 3] = E[:, 0] * 0.5   # rank deficient
        u = O.optimize_gate(E, haar(4, rng))
        assert np.abs(u.conj().T @ u - np.eye(4)).max() < 1e-12
        best = np.real(np.trace(E @ u))
        assert abs(best - O.nuclear_norm(E)) < 1e-12 * max(1.0, O.nuclear_norm(E))
        for _ in range(200):
            W = haar(4, rng)
            assert np.real(np.trace(E @ W)) <= best + 1e-12


def test_update_polar_closed_form():
    """E = P W with P Hermitian positive definite and W unitary: the maximiser
    is W^dagger (Re Tr(P W W^dagger) = Tr P = sum of singular values)."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        W = haar(4, rng)
        A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        P = A @ A.conj().T + 0.1 * np.eye(4)
        u = O.optimize_gate(P @ W, haar(4, rng))
        np.testing.assert_allclose(u, W.conj().T, atol=1e-12)
        # scaled unitary environment: E = c * w^dagger -> u = w
        w = haar(4, rng)
        np.testing.assert_allclose(O.optimize_gate(3.7 * w.conj().T, haar(4, rng)), w, atol=1e-13)


def test_beta_limits():
    rng = np.random.default_rng(5)
    E = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    u0 = haar(4, rng)
    np.testing.assert_allclose(O.optimize_gate(E, u0, beta=1.0), u0, atol=1e-13)   # no update
    np.testing.assert_allclose(O.optimize_gate(E, u0, beta=0.0), O.optimize_gate(E, haar(4, rng)), atol=1e-14)
    np.testing.assert_array_equal(O.optimize_gate(np.zeros((4, 4)), u0), u0)       # zero env keeps gate


def test_single_gate_covering_all_qubits():
    """n = k = 2, one gate: E = V^dagger, the update returns V, cost 0."""
    V = haar(4)
    u0 = haar(4)
    E = O.environment(V, [u0], [(0, 1)], 2, 0)
    np.testing.assert_allclose(E, V.conj().T, atol=1e-15)
    res = O.instantiate(V, u0[None, None], [(0, 1)], 2, tol=1e-12, opt=O.Options(max_iter=3))
    assert res.costs[0] < 1e-14 and res.sweeps == 1
    np.testing.assert_allclose(res.gates[0], V, atol=1e-13)
    # reversed location: the gate equals SWAP V SWAP
    res = O.instantiate(V, u0[None, None], [(1, 0)], 2, tol=1e-12, opt=O.Options(max_iter=3))
    sw = np.eye(4)[[0, 2, 1, 3]]
    np.testing.assert_allclose(res.gates[0], sw @ V @ sw, atol=1e-13)


def test_product_target_one_sweep():
    """V = a (x) b with gates on (0,1) and (2,3): one sweep reaches cost 0
    (closed form: each update is the polar factor of a scaled unitary)."""
    rng = np.random.default_rng(3)
    a, b = haar(4, rng), haar(4, rng)
    V = np.kron(a, b)
    init = rand_gates(2, rng)
    res = O.instantiate(V, init[None], [(0, 1), (2, 3)], 4, tol=1e-13, opt=O.Options(max_iter=5))
    assert res.sweeps == 1 and res.costs[0] < 1e-13
    C = O.circuit_unitary(res.gates, [(0, 1), (2, 3)], 4)
    assert abs(abs(np.trace(V.conj().T @ C)) - 16) < 1e-12


# ---------------------------------------------------------------- sweep invariants

def test_fixed_point_of_own_circuit():
    """Init gates = the target's gates: cost 0, E_g = 2^(n-2) u_g^dagger, and a
    sweep leaves every gate unchanged."""
    pr = I.config2(n_starts=1)
    n = pr.n
    assert O.cost(pr.target, pr.target_gates, pr.locs, n) < 1e-14
    for g in (0, 7, pr.n_gates - 1):
        E = O.environment(pr.target, pr.target_gates, pr.locs, n, g)
        np.testing.assert_allclose(E, (1 << (n - 2)) * pr.target_gates[g].conj().T, atol=1e-12)
    new = O.sweep_definition(pr.target, pr.target_gates, pr.locs, n)
    np.testing.assert_allclose(new, pr.target_gates, atol=1e-12)


@pytest.mark.parametrize("n,p", [(3, 4), (4, 7), (5, 9)])
def test_sweep_monotone_turnaround_and_frobenius(n, p):
    V, gates, locs = _problem(n, p)
    N = 1 << n
    rec = []
    new = O.sweep_definition(V, gates, locs, n, record=rec)
    T0 = O.overlap(V, O.circuit_unitary(gates, locs, n))
    prev = abs(T0)
    for (g, half, E, u, T) in rec:
        assert abs(T) >= prev - 1e-13 * N             # never decreases (Sec. III-A)
        assert abs(T.imag) <= 1e-12 * N and T.real >= 0   # real after a beta=0 update
        assert np.abs(u.conj().T @ u - np.eye(4)).max() < 1e-12
        prev = abs(T)
    # turnaround: the first update of the second half sees the last env of the first half
    first_half_last = rec[p - 1]
    second_first = rec[p]
    assert first_half_last[0] == second_first[0] == 0
    np.testing.assert_allclose(second_first[3], first_half_last[3], atol=1e-12)
    # Frobenius identity after the sweep: ||C - V||^2 = 2 N Delta
    C = O.circuit_unitary(new, locs, n)
    delta = 1 - abs(O.overlap(V, C)) / N
    assert abs(O.frobenius_distance_sq(V, C) - 2 * N * delta) < 1e-12 * N


@pytest.mark.parametrize("n,p,S", [(3, 5, 2), (5, 8, 3), (7, 6, 2)])
def test_builder_mode_equals_definition_mode(n, p, S):
    """Alg. 1's circuit tensor gives the same environments and gates as the
    from-scratch definition, update by update."""
    rng = np.random.default_rng(100 + n)
    V, _, locs = _problem(n, p, rng)
    starts = np.stack([rand_gates(p, rng) for _ in range(S)])
    b = O.BuilderOracle(V, starts, locs, n)
    recb = []
    b.sweep(record=recb)
    b.sweep(record=recb)
    for s in range(S):
        recd = []
        g1 = O.sweep_definition(V, starts[s], locs, n, record=recd)
        O.sweep_definition(V, g1, locs, n, record=recd)
        assert len(recd) == len(recb)
        for (gd, hd, Ed, ud, Td), (gb, hb, Eb, ub, Tb) in zip(recd, recb):
            assert (gd, hd) == (gb, hb)
            np.testing.assert_allclose(Eb[s], Ed, atol=1e-12 * (1 << n))
            np.testing.assert_allclose(ub[s], ud, atol=1e-11)
            assert abs(Tb[s] - Td) < 1e-11 * (1 << n)


# ---------------------------------------------------------------- termination

def test_plateau_readings():
    opt = O.Options()
    hist = [np.array([1.0]), np.array([0.5])]
    assert not O.qfactor_oracle._plateau_flags(hist, 1, opt)[0]
    hist = [np.array([0.5]), np.array([0.5 - 0.5 * 0.9e-5])]       # relative gain < 1e-5
    assert O.qfactor_oracle._plateau_flags(hist, 1, opt)[0]
    hist = [np.array([0.5]), np.array([0.5 - 0.5 * 1.1e-5])]       # relative gain > 1e-5
    assert not O.qfactor_oracle._plateau_flags(hist, 1, opt)[0]
    # long plateau: 100 sweeps that together gain less than 10 %
    c = [np.array([1.0 * (0.9991 ** k)]) for k in range(101)]
    assert O.qfactor_oracle._plateau_flags(c, 100, opt)[0]
    c = [np.array([1.0 * (0.998 ** k)]) for k in range(101)]
    assert not O.qfactor_oracle._plateau_flags(c, 100, opt)[0]
    # tests switched off
    off = O.Options(diff_tol_r=0.0, long_diff_count=0)
    hist = [np.array([0.5]), np.array([0.5])]
    assert not O.qfactor_oracle._plateau_flags(hist, 1, off)[0]


def test_multistart_any_converged_stops_and_best_start():
    pr = I.config1()
    # start 1 is the target's own gates -> converges in the first sweep
    init = np.stack([pr.init_gates[0], pr.target_gates])
    res = O.instantiate(pr.target, init, pr.locs, pr.n, tol=1e-10, opt=O.Options(max_iter=50))
    assert res.status == O.STATUS_CONVERGED and res.sweeps == 1 and res.best_start == 1


def test_max_iter_and_gauge_invariant_comparison():
    pr = I.config1()
    res = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-10,
                        opt=O.Options(max_iter=7, diff_tol_r=0.0, long_diff_count=0))
    assert res.status == O.STATUS_MAX_ITER and res.sweeps == 7 and res.history.shape == (8, 1)
    assert np.all(np.diff(res.history[:, 0]) <= 1e-14)
    # two different converged solutions realise the same unitary up to phase
    conv = []
    for s in range(12):
        init = I.haar_gates(I.rng_for(1, 1, 1000 + s), 4)[None]
        r = O.instantiate(pr.target, init, pr.locs, pr.n, tol=1e-10,
                          opt=O.Options(max_iter=300, diff_tol_r=0.0, long_diff_count=0))
        if r.status == O.STATUS_CONVERGED:
            conv.append(O.circuit_unitary(r.gates, pr.locs, pr.n))
        if len(conv) == 2:
            break
    assert len(conv) == 2
    assert abs(np.trace(conv[0].conj().T @ conv[1])) / 8 >= 1 - 4e-10


def test_nan_start_is_frozen():
    pr = I.config1()
    bad = pr.init_gates[0].copy()
    bad[2, 1, 1] = np.nan
    init = np.stack([bad, pr.target_gates])
    res = O.instantiate(pr.target, init, pr.locs, pr.n, tol=1e-10, opt=O.Options(max_iter=5))
    assert res.best_start == 1 and res.status == O.STATUS_CONVERGED and not np.isfinite(res.costs[0])


@pytest.mark.parametrize("cfg,n_starts", [(45, 3), (49, 4)])
def test_multistart_waits_for_every_plateau_and_plateaued_starts_keep_sweeping(cfg, n_starts):
    """Sec. IV-A: with parallel multistarts the plateau stop is taken only when
    every start has hit a plateau.  Sec. V-A: a start whose plateau test has
    fired keeps iterating with the others.  Starts are independent runs in
    lockstep, so the job's length is the longest solo plateau sweep, and each
    start's cost column equals its own run for that many sweeps with the
    plateau tests switched off.  A start that has hit a plateau stays counted
    as plateaued even when its test stops firing at a later sweep (config
    49: counting only the starts whose test fires in the current sweep would
    run to sweep 95).  Config 45's starts plateau at sweeps 35, 7 and 13;
    config 49's at 13, 10, 12 and 22."""
    n, locs, V, init = I.unreachable_problem(cfg, n_starts)
    S = n_starts
    solo = [O.instantiate(V, init[s], locs, n, tol=1e-10) for s in range(S)]
    ks = [r.sweeps for r in solo]
    assert all(r.status == O.STATUS_PLATEAU for r in solo)
    assert min(ks) + 5 < max(ks)  # the case is staggered
    K = max(ks)
    fixed = [O.instantiate(V, init[s], locs, n, tol=1e-10,
                           opt=O.Options(max_iter=K, diff_tol_r=0.0, long_diff_count=0)) for s in range(S)]
    multi = O.instantiate(V, init, locs, n, tol=1e-10)
    assert multi.status == O.STATUS_PLATEAU and multi.sweeps == K
    for s in range(S):
        np.testing.assert_allclose(multi.history[:, s], fixed[s].history[:, 0], rtol=0, atol=1e-13)
        np.testing.assert_allclose(multi.all_gates[s], fixed[s].all_gates[0], rtol=0, atol=1e-11)
    # the earliest plateau's start went on improving after its test fired
    s0 = int(np.argmin(ks))
    assert multi.history[ks[s0], s0] - multi.history[K, s0] > 1e-9
    assert np.abs(multi.all_gates[s0] - solo[s0].all_gates[0]).max() > 1e-9
    assert multi.best_start == int(np.argmin(multi.costs))
    # the same rule in definition mode (no circuit tensor) stops at the same sweep
    dfn = O.instantiate(V, init, locs, n, tol=1e-10, mode="definition")
    assert dfn.sweeps == K and dfn.status == O.STATUS_PLATEAU


def test_reset_iter_rebuilds_the_circuit_tensor_before_the_cost(monkeypatch):
    """Sec. III-A-2 (reset_iter): the circuit tensor accumulates error from the
    apply / un-apply pairs, so every reset_iter sweeps it is recomputed from
    the gates; the cost of that sweep is then read from the fresh tensor.  A
    drift is planted after every sweep (the tensor scaled by 1 + 1e-7: the
    SVD step is scale invariant, so the gates follow the undisturbed
    trajectory and only the tensor's trace is off).  The costs read at
    multiples of reset_iter are then the from-scratch costs; the others carry
    the drift; with resets off every sweep carries it."""
    pr = I.config1()
    orig = O.BuilderOracle.sweep

    def drifting_sweep(self, record=None, active=None):
        orig(self, record, active)
        self.X = self.X * (1.0 + 1e-7)

    monkeypatch.setattr(O.BuilderOracle, "sweep", drifting_sweep)
    kw = dict(max_iter=7, diff_tol_r=0.0, long_diff_count=0)
    ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-300, mode="definition",
                        opt=O.Options(**kw))
    got = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-300, opt=O.Options(reset_iter=3, **kw))
    off = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-300, opt=O.Options(reset_iter=0, **kw))
    np.testing.assert_allclose(got.all_gates, ref.all_gates, rtol=0, atol=1e-12)
    d = np.abs(got.history[:, 0] - ref.history[:, 0])
    for i in range(1, 8):
        if i % 3 == 0:
            assert d[i] <= 1e-13, (i, d[i])
        else:
            assert d[i] > 1e-9, (i, d[i])
    assert np.all(np.abs(off.history[1:, 0] - ref.history[1:, 0]) > 1e-9)
    # drift grows sweep by sweep until a reset clears it
    assert d[2] > d[1] and d[5] > d[4]


def test_builder_with_default_resets_tracks_definition_mode_across_sweep_40():
    """Sec. III-A-2 default reset_iter = 40: over 45 sweeps the circuit tensor
    (reset after sweep 40) and from-scratch environments give the same cost
    history and gates."""
    pr = I.config1()
    kw = dict(max_iter=45, diff_tol_r=0.0, long_diff_count=0)
    b = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-300, opt=O.Options(**kw))
    d = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-300, mode="definition", opt=O.Options(**kw))
    assert b.sweeps == 45 and d.sweeps == 45
    np.testing.assert_allclose(b.history, d.history, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b.all_gates, d.all_gates, rtol=0, atol=1e-10)


def test_default_hyperparameters_match_paper():
    with open(os.path.join(GOLDEN, "default_hyperparameters.json")) as f:
        ref = json.load(f)
    opt = O.Options()
    for k in ("dist_tol", "diff_tol_a", "diff_tol_r", "long_diff_count", "long_diff_r",
              "min_iter", "max_iter", "reset_iter", "beta"):
        assert getattr(opt, k) == ref[k], k


def test_inputs_targets_are_their_own_circuits():
    for pr in (I.config1(), I.config2(n_starts=2)):
        assert O.cost(pr.target, pr.target_gates, pr.locs, pr.n) < 1e-14
        assert pr.init_gates.shape == (pr.n_starts, pr.n_gates, 4, 4)
    assert I.brickwall_locations(6, 6).shape == (15, 2)
    assert I.brickwall_locations(10, 10).shape == (45, 2)
    assert I.brickwall_locations(12, 8).shape == (44, 2)


def test_batched_update_matches_single():
    rng = np.random.default_rng(21)
    E = rng.standard_normal((6, 4, 4)) + 1j * rng.standard_normal((6, 4, 4))
    E[2] = 0.0
    E[4, 1, 1] = np.nan
    U = np.stack([haar(4, rng) for _ in range(6)])
    for beta in (0.0, 0.3):
        B = O.optimize_gate_batched(E, U, beta)
        for s in range(6):
            ref = O.optimize_gate(E[s], U[s], beta)
            if np.all(np.isfinite(ref)):
                np.testing.assert_allclose(B[s], ref, atol=1e-13)
            else:
                assert not np.any(np.isfinite(B[s]))


def test_builder_rows_one_by_one():
    """Rows of G_p ... G_1 V^dagger computed from single basis rows agree with
    the full dense product."""
    n, p = 5, 6
    V, gates, locs = _problem(n, p)
    X = O.circuit_unitary(gates, locs, n, dense=True) @ V.conj().T
    rows = [0, 3, 17, 31]
    np.testing.assert_allclose(O.builder_rows(V, gates, locs, n, rows), X[rows], atol=1e-13)


def test_update_scale_invariance():
    """The maximiser does not depend on a positive scale of the environment,
    down to tiny and up to huge magnitudes; only a zero environment keeps the
    old gate."""
    rng = np.random.default_rng(31)
    E = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    u0 = haar(4, rng)
    ref = O.optimize_gate(E, u0)
    for c in (1e-200, 1e-100, 1e100, 1e200):
        np.testing.assert_allclose(O.optimize_gate(c * E, u0), ref, atol=1e-13)
        np.testing.assert_allclose(O.optimize_gate_batched((c * E)[None], u0[None])[0], ref, atol=1e-13)
    np.testing.assert_array_equal(O.optimize_gate(1e-305 * E, u0), u0)


# ---------------------------------------------------------------- gradients

@pytest.mark.parametrize("n,p", [(2, 1), (2, 3), (3, 4)])
def test_cost_gradient_is_brute_force_derivative(n, p):
    """Central differences of the cost (dense circuit product) over the real
    and imaginary part of every gate entry."""
    rng = np.random.default_rng(900 + 10 * n + p)
    locs = rand_locs(n, p, rng)
    V = haar(1 << n, rng)
    g = rand_gates(p, rng)
    c, G = O.cost_gradient(V, g, locs, n)
    assert abs(c - O.cost(V, g, locs, n)) < 1e-14
    h = 1e-6
    for k in range(p):
        for i in range(4):
            for j in range(4):
                for unit in (1.0, 1j):
                    gp, gm = g.copy(), g.copy()
                    gp[k, i, j] += h * unit
                    gm[k, i, j] -= h * unit
                    fd = (O.cost(V, gp, locs, n) - O.cost(V, gm, locs, n)) / (2 * h)
                    an = G[k, i, j].real if unit == 1.0 else G[k, i, j].imag
                    assert abs(fd - an) < 1e-8, (k, i, j, unit)


def test_cost_gradient_matches_torch_autograd_convention():
    """The packed gradient equals what torch's autograd accumulates for complex
    leaves (x-derivative + 1j y-derivative) on an independent dense torch
    construction of the cost (Kronecker products, n = 3)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(910)
    locs = [(0, 1), (1, 2), (0, 1)]
    V = haar(8, rng)
    g = rand_gates(3, rng)
    us = [torch.tensor(g[k], dtype=torch.complex128, requires_grad=True) for k in range(3)]
    I2 = torch.eye(2, dtype=torch.complex128)
    C = torch.eye(8, dtype=torch.complex128)
    for u, loc in zip(us, locs):
        M = torch.kron(u, I2) if loc == (0, 1) else torch.kron(I2, u)
        C = M @ C
    L = 1.0 - torch.abs(torch.trace(torch.tensor(V).conj().T @ C)) / 8
    L.backward()
    c, G = O.cost_gradient(V, g, locs, 3)
    assert abs(float(L.detach()) - c) < 1e-14
    for k in range(3):
        assert np.abs(us[k].grad.numpy() - G[k]).max() < 1e-13


def test_gradient_flat_along_gate_phase():
    """A global phase on one gate leaves |Tr| unchanged: Re Tr(G^dagger i u) = 0."""
    rng = np.random.default_rng(920)
    n, p = 3, 5
    locs = rand_locs(n, p, rng)
    V = haar(8, rng)
    g = rand_gates(p, rng)
    _, G = O.cost_gradient(V, g, locs, n)
    for k in range(p):
        assert abs(np.real(np.vdot(G[k], 1j * g[k]))) < 1e-14


def test_riemannian_gradient_vanishes_at_solution():
    """At the global minimum (target = own circuit) every tangent direction
    u (iK), K Hermitian, has zero derivative; away from it some does not."""
    rng = np.random.default_rng(930)
    n, p = 3, 4
    locs = rand_locs(n, p, rng)
    g = rand_gates(p, rng)
    V = O.circuit_unitary(g, locs, n)
    basis = [np.eye(4, dtype=np.complex128)] + list(O.PAULI2)
    c, G = O.cost_gradient(V, g, locs, n)
    assert c < 1e-14
    assert max(abs(np.real(np.vdot(G[k], g[k] @ (1j * K)))) for k in range(p) for K in basis) < 1e-14
    g2 = rand_gates(p, rng)
    _, G2 = O.cost_gradient(V, g2, locs, n)
    assert max(abs(np.real(np.vdot(G2[k], g2[k] @ (1j * K)))) for k in range(p) for K in basis) > 1e-3


def test_su4_closed_forms():
    """exp(i t P) = cos t I + i sin t P for a Pauli product P (P^2 = I);
    theta = 0 gives I; every gate is unitary with determinant 1."""
    rng = np.random.default_rng(940)
    for k in range(15):
        t = float(rng.uniform(-3, 3))
        th = np.zeros(15)
        th[k] = t
        U = O.su4_gate(th)
        assert np.abs(U - (np.cos(t) * np.eye(4) + 1j * np.sin(t) * O.PAULI2[k])).max() < 1e-14
    assert np.abs(O.su4_gate(np.zeros(15)) - np.eye(4)).max() == 0
    th = rng.normal(size=(6, 15))
    U = O.su4_gate(th)
    for u in U:
        assert np.abs(u.conj().T @ u - np.eye(4)).max() < 1e-13
        assert abs(np.linalg.det(u) - 1) < 1e-13
    # the 15 Pauli products are orthogonal, Hermitian and traceless
    P = O.PAULI2
    assert np.abs(np.einsum("aij,bji->ab", P, P) - 4 * np.eye(15)).max() == 0
    assert np.abs(P - np.conj(np.swapaxes(P, -1, -2))).max() == 0


def test_su4_theta_gradient_finite_differences():
    rng = np.random.default_rng(950)
    th = rng.normal(size=(3, 15))
    G = rng.normal(size=(3, 4, 4)) + 1j * rng.normal(size=(3, 4, 4))
    d = O.su4_theta_gradient(th, G)
    h = 1e-6
    for i in range(3):
        for k in range(15):
            tp, tm = th[i].copy(), th[i].copy()
            tp[k] += h
            tm[k] -= h
            fd = (np.real(np.vdot(G[i], O.su4_gate(tp))) - np.real(np.vdot(G[i], O.su4_gate(tm)))) / (2 * h)
            assert abs(fd - d[i, k]) < 1e-8, (i, k)


def test_param_cost_gradient_finite_differences():
    rng = np.random.default_rng(960)
    n, p = 3, 3
    locs = rand_locs(n, p, rng)
    V = haar(8, rng)
    th = rng.normal(size=(p, 15))
    c, d = O.param_cost_gradient(V, th, locs, n)
    h = 1e-6
    for g in range(p):
        for k in range(15):
            tp, tm = th.copy(), th.copy()
            tp[g, k] += h
            tm[g, k] -= h
            fd = (O.cost(V, O.su4_gate(tp), locs, n) - O.cost(V, O.su4_gate(tm), locs, n)) / (2 * h)
            assert abs(fd - d[g, k]) < 1e-8, (g, k)


# ----------------------------------------------------------------- gate kinds

CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], np.complex128)


def dense_single(g, q, n):
    """I (x) g (x) I on qubit q (qubit 0 most significant), by Kronecker products."""
    return np.kron(np.kron(np.eye(1 << q), g), np.eye(1 << (n - q - 1)))


@pytest.mark.parametrize("q,partner", [(0, 1), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_single_qubit_kind_embedding(q, partner):
    """A single-qubit gate stored as g (x) I on (q, partner) is the gate g on
    qubit q, whatever the partner."""
    rng = np.random.default_rng(1000 + 10 * q + partner)
    g = haar(2, rng)
    n = 3
    X = haar(8, rng)
    got = O.apply_left(X, np.kron(g, np.eye(2)), (q, partner), n)
    assert np.abs(got - dense_single(g, q, n) @ X).max() < 1e-14


def test_partner_trace_identity():
    rng = np.random.default_rng(1010)
    for _ in range(5):
        E = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        g = haar(2, rng)
        E2 = np.array([[sum(E[2 * a + c, 2 * b + c] for c in range(2)) for b in range(2)] for a in range(2)])
        assert abs(np.trace(E @ np.kron(g, np.eye(2))) - np.trace(E2 @ g)) < 1e-13


def test_kind_updates_are_maximisers():
    """The U(2) update attains the nuclear norm of M2 and beats Haar U(2)
    trials; the Rz and GPI updates attain the maximum of a dense grid over
    their angle; the fixed kind returns the gate unchanged."""
    rng = np.random.default_rng(1020)
    ts = np.linspace(-np.pi, np.pi, 200001)
    for _ in range(4):
        E = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        u_old = np.kron(haar(2, rng), np.eye(2))
        E2 = np.array([[E[2 * a, 2 * b] + E[2 * a + 1, 2 * b + 1] for b in range(2)] for a in range(2)])
        val = lambda u: np.real(np.trace(E @ u))  # noqa: E731
        u2 = O.optimize_gate_kind(E, u_old, O.KIND_U2)
        assert abs(val(u2) - np.sum(np.linalg.svd(E2, compute_uv=False))) < 1e-12
        assert all(val(u2) >= val(np.kron(haar(2, rng), np.eye(2))) - 1e-12 for _ in range(200))
        assert np.abs(u2[::2, 1::2]).max() < 1e-15 and np.abs(u2[::2, ::2] - u2[1::2, 1::2]).max() < 1e-15
        urz = O.optimize_gate_kind(E, u_old, O.KIND_RZ)
        grid = np.real(E2[0, 0]) + np.real(E2[1, 1] * np.exp(1j * ts))
        assert abs(val(urz) - grid.max()) < 1e-9 and val(urz) >= grid.max() - 1e-12
        ugp = O.optimize_gate_kind(E, u_old, O.KIND_GPI)
        grid = np.real(E2[0, 1] * np.exp(1j * ts) + E2[1, 0] * np.exp(-1j * ts))
        assert abs(val(ugp) - grid.max()) < 1e-9 and val(ugp) >= grid.max() - 1e-12
        assert np.array_equal(O.optimize_gate_kind(E, CNOT, O.KIND_FIXED), CNOT)


def mixed_circuit(rng, n):
    """A U3 + CNOT style circuit with every kind: CNOTs (fixed), single-qubit
    U(2), Rz and GPI gates (partner = a neighbour), and one general U(4)."""
    locs, gates, kinds = [], [], []
    for q in range(n):
        locs.append((q, (q + 1) % n))
        gates.append(np.kron(haar(2, rng), np.eye(2)))
        kinds.append(O.KIND_U2)
    for q in range(n - 1):
        locs.append((q, q + 1))
        gates.append(CNOT)
        kinds.append(O.KIND_FIXED)
        locs.append((q + 1, q))
        gates.append(np.kron(O.rz(rng.uniform(-3, 3)), np.eye(2)))
        kinds.append(O.KIND_RZ)
    locs.append((0, n - 1))
    gates.append(np.kron(O.gpi(rng.uniform(-3, 3)), np.eye(2)))
    kinds.append(O.KIND_GPI)
    locs.append((n - 2, n - 1))
    gates.append(haar(4, rng))
    kinds.append(O.KIND_U4)
    return np.array(locs, np.int32), np.stack(gates), np.array(kinds, np.int32)


def test_kinds_builder_equals_definition_and_fixed_stay():
    """With every kind in one circuit, builder mode equals definition mode
    update by update, fixed gates never change, and Re Tr(E u) never
    decreases across an update."""
    rng = np.random.default_rng(1030)
    n = 4
    locs, g0, kinds = mixed_circuit(rng, n)
    V = haar(16, rng)
    rec_d = []
    gd = O.sweep_definition(V, g0, locs, n, record=rec_d, kinds=kinds)
    rec_b = []
    b = O.BuilderOracle(V, g0, locs, n, kinds=kinds)
    b.sweep(record=rec_b)
    assert len(rec_d) == len(rec_b)
    for (gi, h, E, u, T), (gj, hb, Eb, ub, Tb) in zip(rec_d, rec_b):
        assert gi == gj and h == hb
        assert np.abs(E - Eb[0]).max() < 1e-11 and np.abs(u - ub[0]).max() < 1e-10
    for k in np.where(kinds == O.KIND_FIXED)[0]:
        assert np.array_equal(gd[k], g0[k]) and np.array_equal(b.gates[0, k], g0[k])
    cur = [u.copy() for u in g0]
    for gi, h, E, u, T in rec_d:
        assert np.real(np.trace(E @ u)) >= np.real(np.trace(E @ cur[gi])) - 1e-12
        cur[gi] = u


def test_kinds_fixed_point_of_own_circuit():
    """A target built from a mixed-kind circuit is a fixed point: one sweep
    from the true gates keeps the cost at zero."""
    rng = np.random.default_rng(1040)
    n = 3
    locs, g0, kinds = mixed_circuit(rng, n)
    V = O.circuit_unitary(g0, locs, n)
    g1 = O.sweep_definition(V, g0, locs, n, kinds=kinds)
    assert O.cost(V, g1, locs, n) < 1e-13


def test_ms_definition_and_update():
    """MS(f1, f2) equals exp(-i pi/4 sigma_f1 (x) sigma_f2) (matrix exponential
    of the defining Hamiltonian), and the MS update attains the maximum of
    Re Tr(E MS(f1, f2)) over a dense grid of both angles."""
    from scipy.linalg import expm
    rng = np.random.default_rng(1050)
    X = np.array([[0, 1], [1, 0]], np.complex128)
    Y = np.array([[0, -1j], [1j, 0]], np.complex128)
    for _ in range(3):
        f1, f2 = rng.uniform(-3, 3, 2)
        s1 = np.cos(f1) * X + np.sin(f1) * Y
        s2 = np.cos(f2) * X + np.sin(f2) * Y
        assert np.abs(O.ms(f1, f2) - expm(-1j * np.pi / 4 * np.kron(s1, s2))).max() < 1e-14
    f = np.linspace(-np.pi, np.pi, 721)
    F1, F2 = np.meshgrid(f, f, indexing="ij")
    for _ in range(3):
        E = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        u = O.optimize_gate_kind(E, O.ms(0.3, -1.1), O.KIND_MS)
        best = np.real(np.trace(E @ u))
        es, ed = np.exp(1j * (F1 + F2)), np.exp(1j * (F1 - F2))
        grid = (np.real(np.trace(E)) + np.real(-1j * E[3, 0] / es - 1j * E[0, 3] * es)
                + np.real(-1j * E[2, 1] / ed - 1j * E[1, 2] * ed)) / np.sqrt(2.0)
        assert best >= grid.max() - 1e-12 and best - grid.max() < 1e-4
        assert np.abs(u.conj().T @ u - np.eye(4)).max() < 1e-14


# ---------------------------------------------------------------- three-qubit gates
# The method is stated for gates of any size (Sec. III: the environment of a
# gate is the tensor network with that gate removed; Eq. opt_u holds for any
# unitary size).  These pins tie the oracle's k = 3 forms to independent
# constructions.

def triples(n):
    return [(a, b, c) for a in range(n) for b in range(n) for c in range(n) if len({a, b, c}) == 3]


@pytest.mark.parametrize("n", [3, 4, 5])
def test_k3_embedding_apply_and_trace(n):
    """apply_left / apply_right / embed / partial_trace of a three-qubit gate
    against the Kronecker construction u (x) I after qubit swaps, and the
    orientation identity Tr((u (x) I) X) = Tr(E u)."""
    rng = np.random.default_rng(3000 + n)
    X = I.random_builder(rng, 1, n)[0]
    locs = triples(n)
    if n == 5:
        locs = locs[::4] + [(4, 3, 2), (0, 4, 2)]
    for loc in locs:
        u = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
        K = O.embed_kron(u, loc, n)
        np.testing.assert_allclose(O.embed(u, loc, n), K, atol=1e-13)
        np.testing.assert_allclose(O.apply_left(X, u, loc, n), K @ X, atol=1e-12)
        np.testing.assert_allclose(O.apply_right(X, u, loc, n), X @ K, atol=1e-12)
        E = O.partial_trace(X, loc, n)
        np.testing.assert_allclose(E, O.partial_trace_loops(X, loc, n), atol=1e-13)
        assert abs(np.trace(K @ X) - np.trace(E @ u)) < 1e-12


def test_k3_embed_kron_of_adjacent_leading_qubits():
    """For loc = (0, 1, 2) no swap is needed: the operator is u (x) I."""
    rng = np.random.default_rng(3010)
    u = I.haar_unitary(rng, 8)
    np.testing.assert_allclose(O.embed(u, (0, 1, 2), 4), np.kron(u, np.eye(2)), atol=1e-15)
    # a two-qubit gate embedded as a three-qubit one with an identity factor
    v = I.haar_unitary(rng, 4)
    np.testing.assert_allclose(O.embed(np.kron(v, np.eye(2)), (1, 3, 0), 4), O.embed(v, (1, 3), 4), atol=1e-14)


@pytest.mark.parametrize("n,layers", [(4, 3), (5, 4)])
def test_k3_trace_invariant_and_derivative(n, layers):
    """Tr(E_g u_g) = Tr(V^dagger C) for every three-qubit gate, and E_g is
    the exact derivative: T(u_g := e_ji) = E_g[i, j] (dense products)."""
    pr = I.k3_problem(31, n, layers, 1)
    rng = np.random.default_rng(3020 + n)
    V = I.haar_unitary(rng, 1 << n)
    gates = pr.init_gates[0]
    T = O.overlap(V, O.circuit_unitary(gates, pr.locs, n, dense=True))
    for g in range(pr.n_gates):
        E = O.environment(V, gates, pr.locs, n, g)
        assert abs(np.trace(E @ gates[g]) - T) < 1e-12 * (1 << n)
    g = pr.n_gates // 2
    E = O.environment(V, gates, pr.locs, n, g)
    for (i, j) in [(0, 0), (3, 5), (7, 2)]:
        G = gates.copy()
        G[g] = 0.0
        G[g][j, i] = 1.0
        Tij = O.overlap(V, O.circuit_unitary(G, pr.locs, n, dense=True))
        assert abs(Tij - E[i, j]) < 1e-12 * (1 << n)


def test_k3_update_maximises_and_is_unitary():
    """Eq. opt_u for 8 x 8: the result is unitary, attains the nuclear norm
    (von Neumann's trace inequality bound) and beats random unitaries."""
    rng = np.random.default_rng(3030)
    for k in range(6):
        E = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
        if k == 1:
            E[:, 3] = 0.5 * E[:, 0] - 2j * E[:, 6]  # rank 7
        if k == 2:
            E[2, :] = 0.0                           # zero row
        u = O.optimize_gate(E, np.eye(8, dtype=np.complex128))
        assert np.abs(u.conj().T @ u - np.eye(8)).max() < 1e-12
        nn = O.nuclear_norm(E)
        assert abs(np.real(np.trace(E @ u)) - nn) < 1e-12 * nn
        for _ in range(20):
            w = I.haar_unitary(rng, 8)
            assert np.real(np.trace(E @ w)) <= nn + 1e-12


def test_k3_sweep_monotone_and_builder_equals_definition():
    """Per-update monotonicity at beta = 0 (Sec. III-A) and Alg. 1's circuit
    tensor against the from-scratch definition, update by update, for a
    three-qubit-gate circuit with two starts."""
    n = 5
    pr = I.k3_problem(32, n, 4, 2)
    rng = np.random.default_rng(3040)
    V = I.haar_unitary(rng, 1 << n)
    b = O.BuilderOracle(V, pr.init_gates, pr.locs, n)
    recb = []
    b.sweep(record=recb)
    for s in range(2):
        recd = []
        O.sweep_definition(V, pr.init_gates[s], pr.locs, n, record=recd)
        prev = abs(O.overlap(V, O.circuit_unitary(pr.init_gates[s], pr.locs, n)))
        for (gd, hd, Ed, ud, Td), (gb, hb, Eb, ub, Tb) in zip(recd, recb):
            assert (gd, hd) == (gb, hb)
            np.testing.assert_allclose(Eb[s], Ed, atol=1e-12 * (1 << n))
            np.testing.assert_allclose(ub[s], ud, atol=1e-11)
            assert abs(Td) >= prev - 1e-13 * (1 << n)
            prev = abs(Td)


def test_k3_fixed_point_and_convergence():
    """A target built from three-qubit gates: its own gates are a fixed point
    (cost 0, E_g = 2^(n-3) u_g^dagger), and instantiation from Haar starts
    reaches it."""
    n = 4
    pr = I.k3_problem(33, n, 2, 2)
    assert O.cost(pr.target, pr.target_gates, pr.locs, n) < 1e-14
    for g in range(pr.n_gates):
        E = O.environment(pr.target, pr.target_gates, pr.locs, n, g)
        np.testing.assert_allclose(E, (1 << (n - 3)) * pr.target_gates[g].conj().T, atol=1e-12)
    r = O.instantiate(pr.target, pr.init_gates, pr.locs, n, tol=1e-10, opt=O.Options(max_iter=2000))
    assert r.status == O.STATUS_CONVERGED and r.costs[r.best_start] < 1e-10


# ---------------------------------------------------------------- stored trajectories

def test_stored_full_size_trajectories_satisfy_the_invariants():
    """The full-size one-sweep trajectories under tests/golden/ (written by
    make_sweep_trajectories.py from the oracle) obey what the paper fixes:
    every new gate is unitary (Eq. opt_u), after each beta = 0 update the
    trace is real, non-negative and never decreases in modulus (Sec. III-A-1),
    the first update of the second half reproduces the gate just set
    (turnaround of Alg. 1), the trace equals Tr(E u_new) of that update, and
    the stored cost is 1 - |Tr| / N of the last update."""
    gd = np.load(os.path.join(GOLDEN, "n12_brickwall8_sweep1.npz"), allow_pickle=False)
    N, p = 1 << 12, 44
    U, E, T = gd["gate"], gd["env"], gd["trace"]
    assert U.shape == (2 * p, 4, 4) and [tuple(o) for o in gd["order"][:2]] == [(p - 1, 0), (p - 2, 0)]
    eye = np.eye(4)
    for j in range(2 * p):
        assert np.abs(U[j].conj().T @ U[j] - eye).max() < 1e-12
        assert abs(T[j].imag) <= 1e-12 * N and T[j].real >= 0
        assert abs(np.trace(E[j] @ U[j]) - T[j]) <= 1e-11 * N
        if j:
            assert abs(T[j]) >= abs(T[j - 1]) - 1e-12 * N
    np.testing.assert_allclose(U[p], U[p - 1], atol=1e-12)
    assert abs(float(gd["cost1"]) - (1 - abs(T[-1]) / N)) < 1e-12
    assert float(gd["cost1"]) < float(gd["cost0"])
    g10 = np.load(os.path.join(GOLDEN, "n10_brickwall10_s16_sweep1.npz"), allow_pickle=False)
    assert g10["history"].shape == (2, 3) and np.all(g10["history"][1] < g10["history"][0])
    np.testing.assert_allclose(g10["history"][1], g10["costs"], atol=1e-12)
