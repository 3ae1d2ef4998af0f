"""GPU parity of the batched instantiation (qf_instantiate_batch): many small
independent problems, each QFactor with multistarts in lockstep (Sec. IV-A),
in one persistent launch.  Blocks are independent, so every block's result
must equal the oracle's run of that block alone.

Tolerances: complex128 costs and trajectories agree with the oracle to 1e-10
(entries O(1), rounding ~1e-14 per step); returned gates to 1e-8; complex64
runs return FP64 costs that equal the oracle's cost of the returned gates to
1e-12, and unitary gates."""
import numpy as np
import pytest

import oracle as O
import qfinputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C128_TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def mixed_blocks(seed: int, count: int, n_starts: int, reachable_every: int = 2):
    """Blocks of 2, 3 and 4 qubits with 1..9 nearest-neighbour or arbitrary-pair
    gates; every `reachable_every`-th target is built from the block's own
    structure (reachable), the others are Haar-random unitaries."""
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        n = int(rng.integers(2, 5))
        p = int(rng.integers(1, 10))
        if b % 3 == 0:
            locs = I.random_nn_locations(rng, n, p)
        else:
            locs = np.array([rng.choice(n, 2, replace=False) for _ in range(p)], np.int32)
        tg = I.haar_gates(rng, p)
        V = I.circuit_unitary(tg, locs, n) if b % reachable_every == 0 else I.haar_unitary(rng, 1 << n)
        init = np.stack([I.haar_gates(rng, p) for _ in range(n_starts)])
        probs.append(I.Problem(f"b{b}", n, np.asarray(locs, np.int32), tg, V, init))
    return probs


def run_batch(qf, probs, tol, **kw):
    targets = [dev(p.target) for p in probs]
    gates = [dev(p.init_gates) for p in probs]
    bn, go, lf, tf, gf = qf.pack_batch(targets, [p.locs for p in probs], gates)
    return qf.instantiate_batch(bn, go, lf, tf, gf, probs[0].init_gates.shape[0], tol=tol, **kw)


def oracle_opts(**kw):
    o = O.Options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("n_starts", [3, 16])
def test_batch_c128_matches_oracle(qf, n_starts):
    """Mixed n = 2..4 blocks (ragged last group of the queue), complex128,
    capped at 60 sweeps so some blocks stop on max_iter: sweeps, status, best
    start, every start's final cost and gates equal the oracle's."""
    probs = mixed_blocks(20 + n_starts, 11, n_starts)
    res = run_batch(qf, probs, 1e-10, precision=0, max_iter=60)
    g = res.gates
    for b, pr in enumerate(probs):
        ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-10, opt=oracle_opts(max_iter=60))
        assert res.sweeps[b] == ref.sweeps, b
        assert res.status[b] == ref.status, b
        assert np.abs(res.costs[b] - ref.costs).max() <= C128_TOL, b
        assert res.best[b] == int(np.argmin(res.costs[b])), b
        srt = np.sort(ref.costs)
        if n_starts == 1 or srt[1] - srt[0] > 1e-9:
            assert res.best[b] == ref.best_start, b
        got = host(res.block_gates(b))
        assert np.abs(got - ref.all_gates).max() <= 1e-8, b
    assert g.shape[0] == sum(pr.n_gates * n_starts for pr in probs)


def test_batch_c64_fp64_costs(qf):
    """A complex64 request (run on complex128 builders, see
    qf_instantiate_batch): each returned cost is the oracle's cost of the
    returned gates, the gates are unitary, reachable blocks converge, and the
    results are bitwise those of the complex128 request."""
    probs = mixed_blocks(31, 12, 4)
    res = run_batch(qf, probs, 1e-8, precision=1)
    for b, pr in enumerate(probs):
        gb = host(res.block_gates(b))
        for s in range(4):
            c = O.cost(pr.target, gb[s], pr.locs, pr.n)
            assert abs(c - res.costs[b, s]) <= 1e-12, (b, s)
            assert np.abs(np.conj(np.swapaxes(gb[s], -1, -2)) @ gb[s] - np.eye(4)).max() < 1e-12
        assert res.status[b] == (0 if res.costs[b].min() < 1e-8 else res.status[b])
        if b % 2 == 0:
            assert res.status[b] == 0 and res.costs[b, res.best[b]] < 1e-8, b
    r128 = run_batch(qf, probs, 1e-8, precision=0)
    assert np.array_equal(res.costs, r128.costs) and np.array_equal(res.sweeps, r128.sweeps)


def test_batch_one_start_and_tiny(qf):
    """n_starts = 1 (16 blocks per wavefront), a single n = 2 block with one
    gate, and a block whose target is its own initial circuit (cost 0 at
    sweep 0 is not a stop before sweep 1: the oracle runs one sweep)."""
    probs = mixed_blocks(41, 5, 1)
    rng = np.random.default_rng(42)
    g0 = I.haar_gates(rng, 2)
    locs = np.array([[0, 1], [1, 0]], np.int32)
    probs.append(I.Problem("self", 2, locs, g0, I.circuit_unitary(g0, locs, 2), g0[None].copy()))
    res = run_batch(qf, probs, 1e-10, precision=0, max_iter=40)
    for b, pr in enumerate(probs):
        ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-10, opt=oracle_opts(max_iter=40))
        assert res.sweeps[b] == ref.sweeps and res.status[b] == ref.status, b
        assert np.abs(res.costs[b] - ref.costs).max() <= C128_TOL, b


def test_batch_zero_sweeps_returns_initial(qf):
    """max_iter = 0: the gates come back unchanged with their FP64 costs."""
    probs = mixed_blocks(51, 7, 2)
    for prec in (0, 1):
        res = run_batch(qf, probs, 1e-10, precision=prec, max_iter=0)
        for b, pr in enumerate(probs):
            assert res.sweeps[b] == 0 and res.status[b] == O.STATUS_MAX_ITER
            assert np.array_equal(host(res.block_gates(b)), pr.init_gates)
            c = np.array([O.cost(pr.target, pr.init_gates[s], pr.locs, pr.n) for s in range(2)])
            assert np.abs(res.costs[b] - c).max() <= 1e-12


def test_batch_nan_block_isolated(qf):
    """A block with a non-finite target is reported QF_NUMERIC with infinite
    costs; its neighbours in the same wavefront are unaffected."""
    probs = mixed_blocks(61, 6, 4)
    bad = probs[2]
    bad.target = bad.target.copy()
    bad.target[0, 0] = np.nan
    res = run_batch(qf, probs, 1e-10, precision=0, max_iter=30)
    assert res.status[2] == O.STATUS_NUMERIC and np.all(np.isinf(res.costs[2]))
    for b, pr in enumerate(probs):
        if b == 2:
            continue
        ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=1e-10, opt=oracle_opts(max_iter=30))
        assert res.sweeps[b] == ref.sweeps and res.status[b] == ref.status, b
        assert np.abs(res.costs[b] - ref.costs).max() <= C128_TOL, b


def test_batch_deterministic_and_reusable_workspace(qf):
    probs = mixed_blocks(71, 9, 3)
    r1 = run_batch(qf, probs, 1e-8, precision=1)
    r2 = run_batch(qf, probs, 1e-8, precision=1)
    assert np.array_equal(r1.costs, r2.costs) and np.array_equal(r1.sweeps, r2.sweeps)
    assert torch.equal(r1.gates, r2.gates)


def test_batch_invalid_arguments(qf):
    from paper_2306_08152_amd import QfError
    probs = mixed_blocks(81, 3, 2)
    targets = [dev(p.target) for p in probs]
    gates = [dev(p.init_gates) for p in probs]
    bn, go, lf, tf, gf = qf.pack_batch(targets, [p.locs for p in probs], gates)
    bad_n = bn.copy()
    bad_n[0] = 5
    with pytest.raises(QfError):
        qf.instantiate_batch(bad_n, go, lf, tf, gf, 2)
    with pytest.raises(QfError):
        qf.instantiate_batch(bn, go, lf, tf, gf, 17)
    bad_go = go.copy()
    bad_go[2] = bad_go[1]
    with pytest.raises(QfError):
        qf.instantiate_batch(bn, bad_go, lf, tf, gf, 2)
    bad_l = lf.copy()
    bad_l[0, 0] = bn[0]
    with pytest.raises(QfError):
        qf.instantiate_batch(bn, go, bad_l, tf, gf, 2)


@pytest.mark.slow
@pytest.mark.parametrize("precision", [1, 0])
def test_batch_full_size_sampled(qf, precision):
    """The full 4096-block x 8-start workload in one launch; a sample of
    blocks (both sizes, first and last in the queue) is re-run by the oracle
    alone.  complex128: identical trajectories; complex64: FP64 costs of the
    returned gates and the same convergence outcome."""
    probs = I.config4_blocks()
    res = run_batch(qf, probs, I.C4["tol"], precision=precision)
    assert set(np.unique(res.status)) <= {0, 1, 2}
    for b in range(len(probs)):
        assert (res.status[b] == 0) == (res.costs[b, res.best[b]] < I.C4["tol"])
    sample = [0, 1, 2047, 2048, 2049, 4095]
    for b in sample:
        pr = probs[b]
        gb = host(res.block_gates(b))
        if precision == 0:
            ref = O.instantiate(pr.target, pr.init_gates, pr.locs, pr.n, tol=I.C4["tol"])
            assert res.sweeps[b] == ref.sweeps and res.status[b] == ref.status, b
            assert np.abs(res.costs[b] - ref.costs).max() <= C128_TOL, b
        else:
            for s in range(pr.init_gates.shape[0]):
                assert abs(O.cost(pr.target, gb[s], pr.locs, pr.n) - res.costs[b, s]) <= 1e-12, (b, s)
    frac = float(np.mean(res.status == 0))
    assert frac > 0.5, frac


@pytest.mark.parametrize("n_starts", [3, 8])
def test_batch_launch_shapes_bitwise_equal(qf, n_starts):
    """The tuner of the batched launch (hexes per workgroup, workgroups per
    CU) changes no result: the tuned run and runs forced to each shape give
    bitwise the same costs, sweeps, statuses, best starts and gates, and the
    tuned shape is one of the candidates.  Blocks of uneven gate counts, so
    a workgroup's blocks idle through each other's steps differently in
    every shape."""
    probs = mixed_blocks(91 + n_starts, 40, n_starts)
    cuda = torch.device("cuda")
    qf.set_batch_config(cuda, n_starts, 0)  # tune on this call
    ref = run_batch(qf, probs, 1e-8, precision=0)
    assert (ref.slots, ref.wg_per_cu) in {(16, 1), (8, 1), (8, 2)}
    try:
        for slots, per in ((16, 1), (8, 1), (8, 2)):
            qf.set_batch_config(cuda, n_starts, slots, per)
            r = run_batch(qf, probs, 1e-8, precision=0)
            assert (r.slots, r.wg_per_cu) == (slots, per)
            assert np.array_equal(r.costs, ref.costs)
            assert np.array_equal(r.sweeps, ref.sweeps)
            assert np.array_equal(r.status, ref.status)
            assert np.array_equal(r.best, ref.best)
            assert torch.equal(r.gates, ref.gates)
    finally:
        qf.set_batch_config(cuda, n_starts, 0)


def test_batch_in_place_gates(qf):
    """out_gates == init_gates: the tuner cannot restore trial output, so the
    call takes the default shape untimed; the results equal a run into a
    separate buffer."""
    probs = mixed_blocks(97, 12, 2)
    cuda = torch.device("cuda")
    qf.set_batch_config(cuda, 2, 0)
    targets = [dev(p.target) for p in probs]
    gates = [dev(p.init_gates) for p in probs]
    bn, go, lf, tf, gf = qf.pack_batch(targets, [p.locs for p in probs], gates)
    sep = qf.instantiate_batch(bn, go, lf, tf, gf, 2, tol=1e-8)
    qf.set_batch_config(cuda, 2, 0)
    g_in = gf.clone()
    inp = qf.instantiate_batch(bn, go, lf, tf, g_in, 2, tol=1e-8, out_gates=g_in)
    assert (inp.slots, inp.wg_per_cu) == (16, 1)
    assert torch.equal(inp.gates, sep.gates)
    assert np.array_equal(inp.costs, sep.costs)
    qf.set_batch_config(cuda, 2, 0)
