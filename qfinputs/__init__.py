"""Seeded synthetic workloads for QFactor instantiation (inputs only).

This module draws the random arrays that both the FP64 oracle and the GPU
library consume: Haar-random two-qubit gates, circuit structures (open-chain
brick-walls, random nearest-neighbour blocks), target unitaries built from
seeded gates on the same structure, and random initial gates for the
multistarts.  It holds none of the instantiation method's arithmetic (no
environment, no SVD update, no cost, no termination logic).

The paper evaluates on partitions of real benchmark circuits; those are not
available here, so seeded Haar brick-walls of the same qubit counts and gate
volumes stand in for them (one general U(4) gate is worth about three CNOTs
plus single-qubit gates).

Conventions shared with the rest of the project:
  * n qubits, N = 2**n; qubit 0 is the most significant bit of a row/column
    index; a gate's local index is built from its qubits in the listed order
    (loc[0] is the local most significant bit).
  * gates are listed in time order, so the circuit unitary is
    C = G_p ... G_2 G_1.
  * random streams come from numpy's PCG64 seeded with
    SeedSequence([config_id, role, index]); role 0 = target gates,
    role 1 = initial gates, index = start (or block).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROLE_TARGET = 0
ROLE_INIT = 1
ROLE_STRUCTURE = 2
ROLE_PARAMS = 3


def rng_for(config_id: int, role: int, index: int) -> np.random.Generator:
    """Independent PCG64 stream for (config, role, index)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, role, index])))


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed d x d unitary (QR of a complex Ginibre matrix with the
    phase correction of Mezzadri, 'How to generate random matrices from the
    classical compact groups', Notices AMS 54 (2007))."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    diag = np.diagonal(r)
    ph = diag / np.abs(diag)
    return (q * ph[None, :]).astype(np.complex128)


def haar_gates(rng: np.random.Generator, count: int, d: int = 4) -> np.ndarray:
    """count x d x d stack of Haar unitaries drawn in order from rng."""
    return np.stack([haar_unitary(rng, d) for _ in range(count)]) if count else np.zeros((0, d, d), np.complex128)


def brickwall_locations(n: int, layers: int) -> np.ndarray:
    """Open-chain brick-wall: even layers act on (0,1),(2,3),...; odd layers on
    (1,2),(3,4),...  Returns a (p, 2) int32 array in time order."""
    locs = []
    for layer in range(layers):
        start = 0 if layer % 2 == 0 else 1
        for q in range(start, n - 1, 2):
            locs.append((q, q + 1))
    return np.asarray(locs, dtype=np.int32).reshape(-1, 2)


def random_nn_locations(rng: np.random.Generator, n: int, count: int) -> np.ndarray:
    """count nearest-neighbour pairs (q, q+1) with q uniform in [0, n-2]."""
    qs = rng.integers(0, n - 1, size=count)
    return np.stack([qs, qs + 1], axis=1).astype(np.int32)


def circuit_unitary(gates: np.ndarray, locs: np.ndarray, n: int) -> np.ndarray:
    """Target construction: C = G_p ... G_1 for gates in time order, each on
    k = len(loc) qubits (k = 2 or 3 here).

    Each gate is applied to the running matrix by viewing its row index as n
    binary legs (qubit 0 first) and contracting the gate with the k legs it
    acts on.  Used only to synthesise targets from seeded gates."""
    N = 1 << n
    c = np.eye(N, dtype=np.complex128)
    for u, loc in zip(gates, locs):
        k = len(loc)
        legs = [int(q) for q in loc]
        t = c.reshape((2,) * n + (N,))
        uk = np.asarray(u, np.complex128).reshape((2,) * (2 * k))
        t = np.tensordot(uk, t, axes=(list(range(k, 2 * k)), legs))
        t = np.moveaxis(t, list(range(k)), legs)
        c = np.ascontiguousarray(t.reshape(N, N))
    return c


def brickwall3_locations(n: int, layers: int) -> np.ndarray:
    """Open-chain brick-wall of three-qubit gates: layer l acts on
    (s, s+1, s+2), (s+3, s+4, s+5), ... with s = l mod 3.  Returns a (p, 3)
    int32 array in time order."""
    locs = []
    for layer in range(layers):
        for q in range(layer % 3, n - 2, 3):
            locs.append((q, q + 1, q + 2))
    return np.asarray(locs, dtype=np.int32).reshape(-1, 3)


@dataclass
class Problem:
    """One instantiation problem: target V, structure and initial gates."""

    name: str
    n: int
    locs: np.ndarray            # (p, k) int32, k = 2 (3 for the three-qubit problems)
    target_gates: np.ndarray    # (p, 2^k, 2^k) complex128, the gates V was built from
    target: np.ndarray          # (N, N) complex128 (may be None for huge n until built)
    init_gates: np.ndarray      # (S, p, 2^k, 2^k) complex128
    meta: dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return int(self.locs.shape[0])

    @property
    def n_starts(self) -> int:
        return int(self.init_gates.shape[0])


def make_problem(config_id: int, name: str, n: int, locs: np.ndarray, n_starts: int,
                 build_target: bool = True, block: int = 0) -> Problem:
    """Target from Haar gates (role 0, index=block) on `locs`; init gates for each
    start s from stream (role 1, index=block*65536+s).  Gates act on
    locs.shape[1] qubits (2^k x 2^k Haar unitaries)."""
    locs = np.asarray(locs, np.int32)
    p = int(locs.shape[0])
    d = 1 << int(locs.shape[1])
    tg = haar_gates(rng_for(config_id, ROLE_TARGET, block), p, d)
    init = np.stack([haar_gates(rng_for(config_id, ROLE_INIT, block * 65536 + s), p, d)
                     for s in range(n_starts)]) if n_starts else np.zeros((0, p, d, d), np.complex128)
    target = circuit_unitary(tg, locs, n) if build_target else None
    return Problem(name, n, np.asarray(locs, np.int32), tg, target, init)


# ---------------------------------------------------------------------------
# The five evaluation workloads (sizes, structures, starts).
# ---------------------------------------------------------------------------

C1 = dict(config_id=1, name="n3_p4_c128", n=3, locs=[(0, 1), (1, 2), (0, 1), (1, 2)], starts=1,
          tol=1e-10, max_iter=1000)
C2 = dict(config_id=2, name="n6_brickwall6_s32", n=6, layers=6, starts=32, tol=1e-8)
C3 = dict(config_id=3, name="n10_brickwall10_s16_c64", n=10, layers=10, starts=16, tol=1e-8)
C4 = dict(config_id=4, name="batch4096_n3n4_s8", blocks=4096, starts=8, tol=1e-8)
C5 = dict(config_id=5, name="n12_brickwall8_s1_c64", n=12, layers=8, starts=1, tol=1e-8)


def config1() -> Problem:
    locs = np.asarray(C1["locs"], np.int32)
    return make_problem(C1["config_id"], C1["name"], C1["n"], locs, C1["starts"])


def config2(n_starts: int = C2["starts"]) -> Problem:
    return make_problem(C2["config_id"], C2["name"], C2["n"], brickwall_locations(C2["n"], C2["layers"]), n_starts)


def config3(n_starts: int = C3["starts"], build_target: bool = True) -> Problem:
    return make_problem(C3["config_id"], C3["name"], C3["n"], brickwall_locations(C3["n"], C3["layers"]),
                        n_starts, build_target=build_target)


def config5(n_starts: int = C5["starts"], build_target: bool = True) -> Problem:
    return make_problem(C5["config_id"], C5["name"], C5["n"], brickwall_locations(C5["n"], C5["layers"]),
                        n_starts, build_target=build_target)


def config4_blocks(n_blocks: int = C4["blocks"], n_starts: int = C4["starts"], build_target: bool = True):
    """Batched workload: half 3-qubit, half 4-qubit blocks, each a random
    nearest-neighbour circuit of U{4..20} gates, target from Haar gates on its
    own structure.  Returns a list of Problems."""
    probs = []
    for b in range(n_blocks):
        rs = rng_for(C4["config_id"], ROLE_STRUCTURE, b)
        n = 3 if b < n_blocks // 2 else 4
        count = int(rs.integers(4, 21))
        locs = random_nn_locations(rs, n, count)
        probs.append(make_problem(C4["config_id"], f"block{b}", n, locs, n_starts,
                                  build_target=build_target, block=b))
    return probs


def su4_params(config_id: int, n_starts: int, count: int, scale: float = 1.0) -> np.ndarray:
    """(n_starts, count, 15) Gaussian parameters (standard deviation `scale`)
    for gates exp(i sum_k theta_k P_k); start s draws from stream
    (role 3, index s)."""
    return np.stack([scale * rng_for(config_id, ROLE_PARAMS, s).standard_normal((count, 15))
                     for s in range(n_starts)])


def deletion_problem(config_id: int, n: int, p: int, p_target: int, n_starts: int):
    """Gate-deletion workload: a nearest-neighbour chain of p gates on n
    qubits (gate k on (k mod (n-1), k mod (n-1) + 1)) whose first p - p_target
    gates are identities and the last p_target Haar-random (role 0), the
    target is that circuit's unitary, and a pool of Haar starts (role 1)."""
    locs = np.array([(k % (n - 1), k % (n - 1) + 1) for k in range(p)], np.int32)
    rt = rng_for(config_id, ROLE_TARGET, 0)
    g = np.stack([haar_unitary(rt, 4) if k >= p - p_target else np.eye(4, dtype=np.complex128) for k in range(p)])
    V = circuit_unitary(g, locs, n)
    pool = np.stack([haar_gates(rng_for(config_id, ROLE_INIT, s), p) for s in range(n_starts)])
    return locs, V, g, pool


CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], np.complex128)


def k3_problem(config_id: int, n: int, layers: int, n_starts: int, build_target: bool = True) -> Problem:
    """Three-qubit-gate brick-wall (brickwall3_locations) with Haar U(8) target
    gates and Haar initial gates (make_problem's streams)."""
    return make_problem(config_id, f"k3_n{n}_l{layers}", n, brickwall3_locations(n, layers), n_starts,
                        build_target=build_target)


def u3cx_problem(config_id: int, n: int, layers: int, n_starts: int, build_target: bool = True):
    """The evaluation's U3 + CNOT gate set (kinds: 2 = U(2) variable stored as
    g (x) I on (q, partner), 1 = fixed CNOT): every layer puts a U(2) gate on
    each qubit (partner = the next qubit, the last one's the previous) and
    then CNOTs on (q, q+1) for q of the layer's parity; a final U(2) layer
    closes the circuit.  Target gates Haar (role 0), initial U(2) gates Haar
    per start (role 1).  Returns locs, kinds, target gates, target, init."""
    locs, kinds = [], []
    for layer in range(layers + 1):
        for q in range(n):
            locs.append((q, q + 1 if q + 1 < n else q - 1))
            kinds.append(2)
        if layer == layers:
            break
        for q in range(layer % 2, n - 1, 2):
            locs.append((q, q + 1))
            kinds.append(1)
    locs = np.array(locs, np.int32)
    kinds = np.array(kinds, np.int32)

    def draw(rng):
        return np.stack([np.kron(haar_unitary(rng, 2), np.eye(2)) if k == 2 else CNOT for k in kinds])

    tg = draw(rng_for(config_id, ROLE_TARGET, 0))
    init = np.stack([draw(rng_for(config_id, ROLE_INIT, s)) for s in range(n_starts)])
    target = circuit_unitary(tg, locs, n) if build_target else None
    return locs, kinds, tg, target, init


def unreachable_problem(config_id: int, n_starts: int):
    """Three gates on (0,1),(1,2),(0,1) of 3 qubits against a Haar 8 x 8
    target (role 0) that such a circuit cannot realise, with Haar initial
    gates per start (role 1, index = start).  Every start ends on a plateau,
    at a sweep that depends on its initial gates.  Returns n, locs, target,
    init."""
    n = 3
    locs = np.asarray([(0, 1), (1, 2), (0, 1)], np.int32)
    V = haar_unitary(rng_for(config_id, ROLE_TARGET, 0), 8)
    init = np.stack([haar_gates(rng_for(config_id, ROLE_INIT, s), 3) for s in range(n_starts)])
    return n, locs, V, init


def random_builder(rng: np.random.Generator, n_starts: int, n: int) -> np.ndarray:
    """Generic complex test matrices (S, N, N) with entries ~ CN(0, 1/N)."""
    N = 1 << n
    x = rng.standard_normal((n_starts, N, N)) + 1j * rng.standard_normal((n_starts, N, N))
    return (x / np.sqrt(2.0 * N)).astype(np.complex128)
