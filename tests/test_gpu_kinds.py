"""GPU parity of the gate kinds (Sec. III-A-3 and the U3 + CNOT gate set):
fixed gates, U(2), Rz and GPI single-qubit gates and the Molmer-Sorensen
gate beside general U(4), in the streaming, resident and batched paths,
against the oracle."""
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


def mixed_problem(seed, n, S, reachable=False):
    """Every kind in one circuit: U(2) on each qubit, CNOTs and Rz gates along
    the chain, a GPI, a general U(4) and an MS gate."""
    rng = np.random.default_rng(seed)
    locs, kinds = [], []
    for q in range(n):
        locs.append((q, q + 1 if q + 1 < n else q - 1))
        kinds.append(O.KIND_U2)
    for q in range(n - 1):
        locs.append((q, q + 1))
        kinds.append(O.KIND_FIXED)
        locs.append((q + 1, q))
        kinds.append(O.KIND_RZ)
    locs.append((0, n - 1))
    kinds.append(O.KIND_GPI)
    locs.append((n - 2, n - 1))
    kinds.append(O.KIND_U4)
    locs.append((1, 0))
    kinds.append(O.KIND_MS)
    locs = np.array(locs, np.int32)
    kinds = np.array(kinds, np.int32)

    def draw():
        out = []
        for k in kinds:
            if k == O.KIND_U2:
                out.append(np.kron(I.haar_unitary(rng, 2), np.eye(2)))
            elif k == O.KIND_FIXED:
                out.append(I.CNOT)
            elif k == O.KIND_RZ:
                out.append(np.kron(O.rz(rng.uniform(-3, 3)), np.eye(2)))
            elif k == O.KIND_GPI:
                out.append(np.kron(O.gpi(rng.uniform(-3, 3)), np.eye(2)))
            elif k == O.KIND_MS:
                out.append(O.ms(*rng.uniform(-3, 3, 2)))
            else:
                out.append(I.haar_unitary(rng, 4))
        return np.stack(out)

    tg = draw()
    V = I.circuit_unitary(tg, locs, n) if reachable else I.haar_unitary(rng, 1 << n)
    init = np.stack([draw() for _ in range(S)])
    return locs, kinds, V, init


@pytest.mark.parametrize("n,mode", [(4, 1), (7, 2), (6, 2)])
def test_kinds_match_oracle(qf, n, mode):
    """Trajectory, final costs and gates against the oracle's builder mode
    with the same kinds (complex128), fixed gates bitwise unchanged."""
    locs, kinds, V, init = mixed_problem(2000 + n, n, 2)
    iters = 20 if mode == 1 else 4
    res = qf.instantiate(dev(V), locs, dev(init), tol=1e-12, mode=mode, precision=0, max_iter=iters,
                         diff_tol_r=0.0, long_diff_count=0, history_rows=iters + 1, gate_kinds=kinds)
    ref = O.instantiate(V, init, locs, n, tol=1e-12, opt=O.Options(max_iter=iters, diff_tol_r=0.0,
                                                                     long_diff_count=0), kinds=kinds)
    assert res.sweeps == ref.sweeps == iters
    assert np.abs(res.history - ref.history).max() <= C128_TOL
    assert np.abs(res.costs - ref.costs).max() <= C128_TOL
    got = host(res.all_gates)
    assert np.abs(got - ref.all_gates).max() <= 1e-8
    fixed = kinds == O.KIND_FIXED
    assert np.array_equal(got[:, fixed], init[:, fixed])


def test_kinds_batch_match_oracle(qf):
    probs = []
    for b in range(5):
        n = 3 + (b % 2)
        locs, kinds, V, init = mixed_problem(2100 + b, n, 3)
        probs.append((n, locs, kinds, V, init))
    targets = [dev(p[3]) for p in probs]
    gates = [dev(p[4]) for p in probs]
    bn, go, lf, tf, gf = qf.pack_batch(targets, [p[1] for p in probs], gates)
    kinds_all = np.concatenate([p[2] for p in probs])
    res = qf.instantiate_batch(bn, go, lf, tf, gf, 3, tol=1e-10, precision=0, max_iter=25, gate_kinds=kinds_all)
    for b, (n, locs, kinds, V, init) in enumerate(probs):
        ref = O.instantiate(V, init, locs, n, tol=1e-10, opt=O.Options(max_iter=25), kinds=kinds)
        assert res.sweeps[b] == ref.sweeps and res.status[b] == ref.status, b
        assert np.abs(res.costs[b] - ref.costs).max() <= C128_TOL, b
        assert np.abs(host(res.block_gates(b)) - ref.all_gates).max() <= 1e-8, b


@pytest.mark.parametrize("precision", [0, 1])
def test_u3cx_converges(qf, precision):
    """The U3 + CNOT gate set on n = 5 (3 layers): a reachable target is
    re-instantiated below 1e-8 from Haar U(2) starts; returned costs are the
    oracle's costs of the returned gates; CNOTs are untouched."""
    locs, kinds, tg, V, init = I.u3cx_problem(7, 5, 3, 8)
    res = qf.instantiate(dev(V), locs, dev(init), tol=1e-8, precision=precision, gate_kinds=kinds)
    allg = host(res.all_gates)
    for s in range(8):
        assert abs(O.cost(V, allg[s], locs, 5) - res.costs[s]) <= 1e-12
    assert np.array_equal(allg[:, kinds == 1], init[:, kinds == 1])
    assert res.status == 0 and res.costs[res.best_start] < 1e-8


def test_kinds_invalid(qf):
    from paper_2306_08152_amd import QfError
    locs, kinds, V, init = mixed_problem(2200, 3, 1)
    bad = kinds.copy()
    bad[0] = 9
    with pytest.raises(QfError):
        qf.instantiate(dev(V), locs, dev(init), gate_kinds=bad)
