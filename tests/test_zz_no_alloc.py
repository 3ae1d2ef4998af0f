"""qf_instantiate_noalloc (the variant of qf_instantiate that works in the
library's fixed device workspace and allocates nothing) against
qf_instantiate with a caller workspace, on the same seeded inputs.

Both run the same kernels in the same order, so gates, costs, sweep counts
and status must agree bitwise.  Two calls in a row, the second smaller than
the first, check that nothing the first call left in the shared array
leaks into the second."""
import ctypes

import numpy as np
import pytest

import qfinputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(cfg, n, layers, S):
    locs = I.brickwall_locations(n, layers)
    pr = I.make_problem(cfg, f"noalloc{n}", n, locs, S, build_target=True)
    V = torch.from_numpy(pr.target).to("cuda")
    g = torch.from_numpy(pr.init_gates).to("cuda")
    return pr, V, g


def _same(a, b):
    assert a.sweeps == b.sweeps
    assert a.status == b.status
    assert a.best_start == b.best_start
    assert a.mode_used == b.mode_used
    np.testing.assert_array_equal(a.costs, b.costs)
    np.testing.assert_array_equal(a.gates.cpu().numpy(), b.gates.cpu().numpy())
    np.testing.assert_array_equal(a.all_gates.cpu().numpy(), b.all_gates.cpu().numpy())
    np.testing.assert_array_equal(a.history, b.history)


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_matches_workspace_call_two_calls_shrinking(qf, prec):
    """Streaming n = 8 with 4 starts, then n = 7 with 2 starts, then the
    resident n = 5 with 3 starts: each call of the fixed-workspace entry point
    against qf_instantiate with its own workspace."""
    cases = [(71, 8, 4, 4), (72, 7, 3, 2), (73, 5, 4, 3)]
    for cfg, n, layers, S in cases:
        pr, V, g = _problem(cfg, n, layers, S)
        kw = dict(tol=1e-9, precision=prec, max_iter=25, history_rows=26)
        ref = qf.instantiate(V, pr.locs, g, **kw)
        got = qf.instantiate(V, pr.locs, g, noalloc=True, **kw)
        print(f"noalloc case n={n} S={S} prec={prec}: sweeps={got.sweeps} status={got.status} "
              f"best={got.costs[got.best_start]:.3e}", flush=True)
        _same(ref, got)


def test_noalloc_repeated_call_same_result(qf):
    """The same call twice: the second starts from what the first left in the
    array and must still give bitwise the same outputs."""
    pr, V, g = _problem(74, 7, 4, 3)
    kw = dict(tol=1e-9, precision=1, max_iter=20, history_rows=21)
    a = qf.instantiate(V, pr.locs, g, noalloc=True, **kw)
    b = qf.instantiate(V, pr.locs, g, noalloc=True, **kw)
    _same(a, b)


def test_noalloc_rejects_oversized_problem(qf):
    """n = 11, one start in complex64 needs more than the fixed 64 MiB: the
    call returns QF_EWORKSPACE before any device work."""
    from paper_2306_08152_amd import _native as nat
    lib = nat.load()
    opt = qf.default_options(precision=1)
    need = int(lib.qf_workspace_size(11, 10, 1, ctypes.byref(opt)))
    assert need > nat.QF_NOALLOC_WORKSPACE_BYTES
    locs = I.brickwall_locations(11, 2)
    V = torch.eye(1 << 11, dtype=torch.complex128, device="cuda")
    g = torch.from_numpy(I.haar_gates(I.rng_for(75, 1, 0), len(locs))[None]).to("cuda")
    with pytest.raises(nat.QfError) as ei:
        qf.instantiate(V, locs, g, tol=1e-9, precision=1, max_iter=2, noalloc=True)
    assert ei.value.code == nat.QF_EWORKSPACE
    assert "64" in str(ei.value) or str(nat.QF_NOALLOC_WORKSPACE_BYTES) in str(ei.value)
