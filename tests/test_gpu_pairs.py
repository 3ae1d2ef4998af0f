"""GPU parity of the two-gate updates (one partial trace and one builder pass
for two consecutive gate updates of a sweep): qf_instantiate in streaming
mode against the FP64 oracle, which updates one gate at a time exactly as
Alg. 1 does, and against the library's own one-pass-per-update path.

Covered: gates on disjoint qubits (4-qubit unions) and on a shared qubit
(3-qubit unions), gate locations given in either order, both halves of a
sweep, unions at the lowest and the highest bits, a multi-workgroup partial
trace (n = 11), restricted gate kinds and fixed gates (which are never
paired), and complex64 and complex128 builders (gate_pairs = 2 turns the
two-gate path on for complex128, where it is off by default)."""
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


C128_TOL = 1e-10
C64_TOL = 1e-5


def random_locations(rng, n, p):
    """p gates on random distinct qubit pairs, either order (shared-qubit and
    disjoint neighbours, low and high bits)."""
    out = []
    for _ in range(p):
        a, b = rng.choice(n, size=2, replace=False)
        out.append((int(a), int(b)))
    return np.asarray(out, np.int32)


def _problem(cfg, n, locs, S):
    return I.make_problem(cfg, f"pairs{cfg}", n, locs, S, build_target=True)


def _unit_count(locs, n, kinds=None):
    """Update units per half-sweep under the greedy pairing of consecutive
    gates in processing order (3- or 4-qubit unions, no fixed gate)."""
    p = len(locs)
    total = 0
    for half in range(2):
        order = list(range(p - 1, -1, -1)) if half == 0 else list(range(p))
        k = 0
        while k < p:
            if k + 1 < p:
                f, s = order[k], order[k + 1]
                m = len({*locs[f].tolist(), *locs[s].tolist()})
                fixed = kinds is not None and (kinds[f] == 1 or kinds[s] == 1)
                if m in (3, 4) and not fixed:
                    k += 2
                    total += 1
                    continue
            k += 1
            total += 1
    return total


CASES = [
    # (config id, n, structure, starts)
    (81, 7, "brickwall", 2),
    (82, 8, "random", 3),
    (83, 9, "random", 2),
    (84, 10, "brickwall", 2),
    (85, 11, "random", 1),
]


def _locs(cfg, n, kind):
    if kind == "brickwall":
        return I.brickwall_locations(n, 4)
    return random_locations(np.random.default_rng(cfg), n, 3 * n if n < 10 else 2 * n)


@pytest.mark.parametrize("cfg,n,kind,S", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_pairs_match_oracle(qf, cfg, n, kind, S, precision):
    """Three sweeps of the two-gate path against the oracle's one-gate-at-a-
    time sweeps: cost after every sweep (complex128 to 1e-10, complex64 to
    1e-5), the final FP64 costs, and (complex128) every returned gate."""
    locs = _locs(cfg, n, kind)
    pr = _problem(cfg, n, locs, S)
    sweeps = 3
    res = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), tol=1e-300, mode=2, precision=precision,
                         max_iter=sweeps, diff_tol_r=0.0, long_diff_count=0, history_rows=sweeps + 1, gate_pairs=2)
    ref = O.instantiate(pr.target, pr.init_gates, pr.locs, n, tol=1e-300,
                        opt=O.Options(max_iter=sweeps, diff_tol_r=0.0, long_diff_count=0))
    print(f"pairs cfg={cfg} n={n} prec={precision}: history diff "
          f"{np.abs(res.history - ref.history).max():.2e}", flush=True)
    tol = C128_TOL if precision == 0 else C64_TOL
    assert res.sweeps == sweeps
    assert np.abs(res.history - ref.history).max() <= tol
    assert np.abs(res.costs - ref.costs).max() <= tol
    if precision == 0:
        assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-8
    g = host(res.all_gates)
    eye = np.eye(4)
    assert np.abs(np.conj(np.swapaxes(g, -1, -2)) @ g - eye).max() < 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_pairs_against_single_updates(qf, precision):
    """The same sweeps with and without two-gate updates: complex128 gates
    agree to 1e-11 and costs to 1e-12 (only summation orders differ);
    complex64 costs to 1e-6."""
    pr = _problem(86, 9, random_locations(np.random.default_rng(86), 9, 24), 3)
    kw = dict(tol=1e-300, mode=2, precision=precision, max_iter=4, diff_tol_r=0.0, long_diff_count=0,
              history_rows=5)
    a = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), gate_pairs=2, **kw)
    b = qf.instantiate(dev(pr.target), pr.locs, dev(pr.init_gates), gate_pairs=0, **kw)
    if precision == 0:
        assert np.abs(host(a.all_gates) - host(b.all_gates)).max() <= 1e-11
        assert np.abs(a.history - b.history).max() <= 1e-12
    else:
        assert np.abs(a.history - b.history).max() <= 1e-6


def test_pairs_with_gate_kinds_match_oracle(qf):
    """U3 + CNOT at n = 8: the U(2) variables pair with each other, the fixed
    CNOTs are updated alone; complex128 history and gates against the
    oracle."""
    locs, kinds, _, V, init = I.u3cx_problem(87, 8, 3, 2)
    sweeps = 3
    res = qf.instantiate(dev(V), locs, dev(init), tol=1e-300, mode=2, precision=0, max_iter=sweeps,
                         diff_tol_r=0.0, long_diff_count=0, gate_kinds=kinds, history_rows=sweeps + 1,
                         gate_pairs=2)
    ref = O.instantiate(V, init, locs, 8, tol=1e-300,
                        opt=O.Options(max_iter=sweeps, diff_tol_r=0.0, long_diff_count=0), kinds=kinds)
    assert np.abs(res.history - ref.history).max() <= C128_TOL
    assert np.abs(host(res.all_gates) - ref.all_gates).max() <= 1e-8


@pytest.mark.parametrize("precision", [1, 0])
def test_pass2_tiles_bitwise_equal(qf, precision):
    """Every tiles-per-workgroup count of the two-gate pass (1, 2, 4, 8: the
    complex64 form stages the operands of each workgroup's tiles in LDS by
    their order) gives bitwise the same gates and costs over two sweeps of
    n = 10 with 16 starts, and the first two starts' costs follow the oracle."""
    import torch
    cuda = torch.device("cuda", 0)
    pr = I.config3(n_starts=16)
    sweeps = 2
    kw = dict(tol=1e-300, mode=2, max_iter=sweeps, precision=precision, diff_tol_r=0.0, long_diff_count=0,
              history_rows=sweeps + 1, gate_pairs=2)
    V, g = dev(pr.target), dev(pr.init_gates)
    runs = []
    try:
        for tiles in (1, 2, 4, 8):
            qf.set_pass2_tiles(cuda, precision, 10, tiles)
            runs.append(qf.instantiate(V, pr.locs, g, **kw))
    finally:
        qf.set_pass2_tiles(cuda, precision, 10, 0)
    for r in runs[1:]:
        assert np.array_equal(host(r.all_gates), host(runs[0].all_gates))
        assert np.array_equal(r.costs, runs[0].costs)
    # the oracle on the first two starts (each start's sweeps are independent)
    ref = O.instantiate(pr.target, pr.init_gates[:2], pr.locs, 10, tol=1e-300,
                        opt=O.Options(max_iter=sweeps, diff_tol_r=0.0, long_diff_count=0))
    tol = C128_TOL if precision == 0 else C64_TOL
    assert np.abs(runs[0].history[:, :2] - ref.history).max() <= tol
    with pytest.raises(Exception):
        qf.set_pass2_tiles(cuda, precision, 10, 3)


def test_pairs_timing_counts_units(qf):
    """The timing run counts one pass and one environment launch per update
    unit (a pair or a single gate) and gives bitwise the default schedule's
    results."""
    pr = I.config3(n_starts=4)
    sweeps = 2
    kw = dict(tol=1e-300, max_iter=sweeps, precision=1, diff_tol_r=0.0, long_diff_count=0)
    V, g = dev(pr.target), dev(pr.init_gates)
    a = qf.instantiate(V, pr.locs, g, **kw)
    b = qf.instantiate(V, pr.locs, g, timing=True, **kw)
    assert np.array_equal(host(a.all_gates), host(b.all_gates))
    assert np.array_equal(a.costs, b.costs)
    units = _unit_count(pr.locs, 10)
    assert units < 2 * len(pr.locs)
    assert b.timing["pass_launches"] == units * sweeps
    assert b.timing["env_launches"] == units * sweeps
