"""FP64 CPU oracle for QFactor's instantiation sweep (arXiv 2306.08152).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the GPU library and imports nothing from it; it is written from the paper in
plain NumPy complex128.

What the paper fixes (Sec. III):
  * instantiation maximises |Tr(V^dagger C)| over the gate unitaries, where C
    is the circuit unitary (Sec. II, problem statement);
  * cost Delta = 1 - |Tr(V^dagger C)| / N (Sec. II);
  * every gate enters Tr(V^dagger C) linearly, so Tr(V^dagger C) = Tr(E u_g)
    for an environment matrix E that does not depend on u_g (Sec. III, Eq. cost
    and the text after it);
  * the best unitary for a fixed environment comes from its SVD,
    E = X D Y^dagger  =>  u_new = Y X^dagger (Sec. III-A-1, Eq. opt_u);
  * the sweep updates the gates one by one, in one direction and then back
    (TwoSidedSweep of Alg. 1), and repeats until termination (Sec. III-A-2);
  * beta mixes the old gate into the SVD argument: (1-beta) E + beta u^dagger
    (Sec. III-A-2, Beta).

Readings where the paper is silent or garbled (same list as in the design
notes):
  Q1  qubit 0 is the most significant bit; a gate's local index follows its
      location order (loc[0] = local most significant bit).
  Q2  gates are in time order: C = G_p ... G_1.
  Q3  the circuit tensor starts as V^dagger (it must represent V^dagger U).
  Q4  "ApplyRight" multiplies onto the output legs (left product G X);
      "ApplyLeft" onto the input legs (right product X G).
  Q5  sweep order follows Alg. 1: g = p..1, then g = 1..p.
  Q6  E is defined by Tr(V^dagger C) = Tr(E u_g), i.e. E[i,j] = dT/du_g[j,i].
  Q7  success test: Delta < dist_tol.
  Q8  short plateau: c_{i-1} - c_i <= diff_tol_a + diff_tol_r * c_i
      (active only when diff_tol_a > 0 or diff_tol_r > 0).
  Q9  long plateau (i >= L = long_diff_count > 0):
      c_{i-L} - c_i < long_diff_r * c_{i-L}.
  Q10 no termination test before sweep min_iter.
  Q11 tests run once per sweep on c_i = Delta after sweep i; c_0 is the cost
      of the initial gates; max_iter counts sweeps.
  Q12 builder mode rebuilds the circuit tensor after sweep i when
      i % reset_iter == 0, before c_i is taken.
  Q13 multistarts run in lockstep; stop when any start succeeds, when every
      start has (at some sweep) met a plateau test, or at max_iter; a start
      whose cost is not finite is frozen and counts as plateaued; the result
      is the start with the smallest final cost (lowest index on ties).
  Q15 a zero environment keeps the old gate.

Pins that tie this oracle to the paper and to mathematics (not to itself) are
in tests/test_oracle_pins.py: the fixed point of a target built from the
circuit itself, the trace identity Tr(E u) = Tr(V^dagger C), the environment as
the exact derivative of the trace (brute force), unitarity, local optimality
against random unitaries (von Neumann trace inequality), per-update
monotonicity, the Frobenius identity of Eq. cost, closed-form single-gate and
product-target cases, dense Kronecker embeddings, and builder mode against
definition mode; for the gradient: brute-force central differences, torch's
own autograd on an independent dense construction, the flat gate-phase
direction, the vanishing Riemannian gradient at the global minimum, the
closed form exp(i t P) = cos t I + i sin t P of the parameterised gates, and
finite differences of the parameter chain rule.  Gates may act on any number
k of qubits (2^k x 2^k unitaries; the paper states the method for any gate
size); the three-qubit forms are pinned against Kronecker embeddings after
qubit swaps, brute-force derivatives, the nuclear-norm bound of Eq. opt_u,
builder against definition mode and the fixed point of a target's own gates.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Options", "embed", "embed_kron", "apply_left", "apply_right", "circuit_unitary",
    "overlap", "cost", "partial_trace", "partial_trace_loops", "environment",
    "optimize_gate", "sweep_definition", "BuilderOracle", "instantiate",
    "STATUS_CONVERGED", "STATUS_PLATEAU", "STATUS_MAX_ITER", "STATUS_NUMERIC",
    "nuclear_norm", "frobenius_distance_sq", "optimize_gate_batched", "builder_rows",
    "cost_gradient", "PAULI2", "su4_hermitian", "su4_gate", "su4_theta_gradient", "param_cost_gradient",
    "KIND_U4", "KIND_FIXED", "KIND_U2", "KIND_RZ", "KIND_GPI", "KIND_MS", "optimize_gate_kind", "rz", "gpi",
    "ms",
]

STATUS_CONVERGED = 0
STATUS_PLATEAU = 1
STATUS_MAX_ITER = 2
STATUS_NUMERIC = 3


# ---------------------------------------------------------------------------
# Gate embedding (Sec. III: gate contraction onto the legs it acts on).
# ---------------------------------------------------------------------------

def _local_and_rest(n: int, loc) -> tuple[np.ndarray, np.ndarray]:
    """For every basis index r of n qubits: the gate-local index a(r) formed
    from the bits of the qubits in loc (loc[0] most significant) and rest(r),
    r with those bits cleared."""
    N = 1 << n
    r = np.arange(N)
    k = len(loc)
    a = np.zeros(N, dtype=np.int64)
    rest = r.copy()
    for t, q in enumerate(loc):
        bit = n - 1 - int(q)
        a |= ((r >> bit) & 1) << (k - 1 - t)
        rest &= ~(1 << bit)
    return a, rest


def embed(u: np.ndarray, loc, n: int) -> np.ndarray:
    """Dense N x N operator of gate u on qubits loc (identity elsewhere):
    G[r, c] = u[a(r), a(c)] if rest(r) == rest(c) else 0."""
    a, rest = _local_and_rest(n, loc)
    same = rest[:, None] == rest[None, :]
    return np.where(same, u[a[:, None], a[None, :]], 0.0).astype(np.complex128)


def _swap_qubits_perm(n: int, q1: int, q2: int) -> np.ndarray:
    """Permutation matrix that exchanges qubits q1 and q2."""
    N = 1 << n
    P = np.zeros((N, N), dtype=np.complex128)
    b1, b2 = n - 1 - q1, n - 1 - q2
    for r in range(N):
        x1, x2 = (r >> b1) & 1, (r >> b2) & 1
        s = r & ~(1 << b1) & ~(1 << b2)
        s |= (x1 << b2) | (x2 << b1)
        P[s, r] = 1.0
    return P


def embed_kron(u: np.ndarray, loc, n: int) -> np.ndarray:
    """Textbook construction of the same operator for a gate on k = len(loc)
    qubits: bring loc to the leading positions 0..k-1 with qubit swaps, use
    the Kronecker form u (x) I_{2^(n-k)}, and swap back.  Independent of
    `embed`; used as a pin."""
    k = len(loc)
    N = 1 << n
    # permutation P maps qubit loc[t] -> position t
    P = np.eye(N, dtype=np.complex128)
    order = list(range(n))  # order[pos] = original qubit currently at position pos

    def swap(pos1, pos2):
        nonlocal P
        S = _swap_qubits_perm(n, pos1, pos2)
        P = S @ P
        order[pos1], order[pos2] = order[pos2], order[pos1]

    for t, q in enumerate(loc):
        pq = order.index(int(q))
        if pq != t:
            swap(t, pq)
    core = np.kron(u, np.eye(N >> k, dtype=np.complex128))
    return P.conj().T @ core @ P


# ---------------------------------------------------------------------------
# Structured application (same operator, applied by leg contraction).
# ---------------------------------------------------------------------------

def apply_left(X: np.ndarray, u: np.ndarray, loc, n: int) -> np.ndarray:
    """G X for G = u on loc (a gate on k = len(loc) qubits, u of side 2^k).
    X is (N, M) (any number M of columns) or carries one leading batch axis
    (S, N, M); u may then be (S, 2^k, 2^k) (one gate per batch entry) or
    (2^k, 2^k)."""
    M = X.shape[-1]
    k = len(loc)
    d = 1 << k
    batch = X.shape[:-2]
    if u.ndim == 2:
        u = np.broadcast_to(u, batch + (d, d))
    lt = [chr(ord('a') + i) for i in range(n)]
    new = [chr(ord('A') + t) for t in range(k)]  # output legs of the gate
    z = 'Z' if batch else ''
    xin = z + ''.join(lt) + 'Y'
    out_l = list(lt)
    for t, q in enumerate(loc):
        out_l[int(q)] = new[t]
    uin = z + ''.join(new) + ''.join(lt[int(q)] for q in loc)
    xo = z + ''.join(out_l) + 'Y'
    Xr = X.reshape(batch + (2,) * n + (M,))
    ur = u.reshape(batch + (2,) * (2 * k))
    out = np.einsum(f"{uin},{xin}->{xo}", ur, Xr, optimize=True)
    return out.reshape(X.shape)


def apply_right(X: np.ndarray, u: np.ndarray, loc, n: int) -> np.ndarray:
    """X G for G = u on loc (gate size and batch rules as apply_left)."""
    N = 1 << n
    k = len(loc)
    d = 1 << k
    batch = X.shape[:-2]
    if u.ndim == 2:
        u = np.broadcast_to(u, batch + (d, d))
    lt = [chr(ord('a') + i) for i in range(n)]
    new = [chr(ord('A') + t) for t in range(k)]  # input legs after the product
    z = 'Z' if batch else ''
    xin = z + 'Y' + ''.join(lt)
    out_l = list(lt)
    for t, q in enumerate(loc):
        out_l[int(q)] = new[t]
    uin = z + ''.join(lt[int(q)] for q in loc) + ''.join(new)
    xo = z + 'Y' + ''.join(out_l)
    Xr = X.reshape(batch + (N,) + (2,) * n)
    ur = u.reshape(batch + (2,) * (2 * k))
    out = np.einsum(f"{xin},{uin}->{xo}", Xr, ur, optimize=True)
    return out.reshape(X.shape)


def circuit_unitary(gates, locs, n: int, dense: bool = False) -> np.ndarray:
    """C = G_p ... G_1 (gates in time order, Q2)."""
    N = 1 << n
    C = np.eye(N, dtype=np.complex128)
    for u, loc in zip(gates, locs):
        C = embed(u, loc, n) @ C if dense else apply_left(C, u, loc, n)
    return C


def builder_rows(V: np.ndarray, gates, locs, n: int, rows) -> np.ndarray:
    """Selected rows of the circuit tensor X = G_p ... G_1 V^dagger, one by
    one: row r of C is (C^T e_r)^T with C^T = G_1^T ... G_p^T, and the row of
    X is that row times V^dagger."""
    N = 1 << n
    E = np.zeros((N, len(rows)), dtype=np.complex128)
    for k, r in enumerate(rows):
        E[r, k] = 1.0
    for u, loc in reversed(list(zip(gates, locs))):
        E = apply_left(E, np.asarray(u).T, loc, n)
    return E.T @ V.conj().T


def overlap(V: np.ndarray, C: np.ndarray) -> complex:
    """T = Tr(V^dagger C) (Sec. II)."""
    return complex(np.vdot(V, C))


def cost(V: np.ndarray, gates, locs, n: int) -> float:
    """Delta = 1 - |Tr(V^dagger C)| / N (Sec. II)."""
    C = circuit_unitary(gates, locs, n)
    return 1.0 - abs(overlap(V, C)) / (1 << n)


# ---------------------------------------------------------------------------
# Environment (Sec. III, Fig. tensors; Q6).
# ---------------------------------------------------------------------------

def partial_trace_loops(X: np.ndarray, loc, n: int) -> np.ndarray:
    """E[i, j] = sum over rest of X[(i, rest), (j, rest)] written as explicit
    loops (small n only)."""
    N = 1 << n
    bits = [n - 1 - int(q) for q in loc]
    k = len(loc)
    d = 1 << k
    E = np.zeros((d, d), dtype=np.complex128)
    for r in range(N):
        if any((r >> b) & 1 for b in bits):
            continue  # r enumerates 'rest' values: local bits cleared
        for i in range(d):
            ri = r
            for t, b in enumerate(bits):
                ri |= ((i >> (k - 1 - t)) & 1) << b
            for j in range(d):
                cj = r
                for t, b in enumerate(bits):
                    cj |= ((j >> (k - 1 - t)) & 1) << b
                E[i, j] += X[ri, cj]
    return E


def partial_trace(X: np.ndarray, loc, n: int) -> np.ndarray:
    """Same partial trace by index contraction (gate on k = len(loc)
    qubits); X may carry one batch axis."""
    batch = X.shape[:-2]
    k = len(loc)
    lt = [chr(ord('a') + i) for i in range(n)]
    new = [chr(ord('A') + t) for t in range(k)]
    col = list(lt)
    for t, q in enumerate(loc):
        col[int(q)] = new[t]
    z = 'Z' if batch else ''
    sub = z + ''.join(lt) + ''.join(col)
    outs = z + ''.join(lt[int(q)] for q in loc) + ''.join(new)
    Xr = X.reshape(batch + (2,) * (2 * n))
    E = np.einsum(f"{sub}->{outs}", Xr, optimize=True)
    return E.reshape(batch + (1 << k, 1 << k))


def environment(V: np.ndarray, gates, locs, n: int, g: int) -> np.ndarray:
    """From-scratch environment of gate g (0-based):
    A_g = (G_{g-1} ... G_1) V^dagger (G_p ... G_{g+1}),  E_g = Tr_rest(A_g),
    so that Tr(E_g u_g) = Tr(A_g G_g) = Tr(V^dagger C)."""
    N = 1 << n
    A = V.conj().T.copy()
    R = np.eye(N, dtype=np.complex128)
    for h in range(g + 1, len(gates)):
        R = apply_left(R, gates[h], locs[h], n)  # R = G_h ... G_{g+1}
    A = A @ R
    for h in range(0, g):
        A = apply_left(A, gates[h], locs[h], n)  # left factor G_{g-1} ... G_1
    return partial_trace(A, locs[g], n)


# ---------------------------------------------------------------------------
# Gate update (Sec. III-A-1, Eq. opt_u; beta of Sec. III-A-2).
# ---------------------------------------------------------------------------

def optimize_gate(E: np.ndarray, u_old: np.ndarray, beta: float = 0.0) -> np.ndarray:
    """argmax over unitary u of Re Tr(M u) for M = (1-beta) E + beta u_old^dagger:
    SVD M = X D Y^dagger gives u = Y X^dagger.  A zero M (largest entry below
    1e-300) keeps u_old (Q15)."""
    M = (1.0 - beta) * E + beta * u_old.conj().T
    if not np.all(np.isfinite(M)):
        return np.full_like(u_old, np.nan)
    scale = np.max(np.abs(M))
    if scale < 1e-300:
        return u_old.copy()
    # the maximiser is unchanged by a positive scaling of M: normalise first
    Xs, _, Yh = np.linalg.svd(M / scale)
    return Yh.conj().T @ Xs.conj().T


# ---------------------------------------------------------------------------
# Gate kinds (Sec. III-A-3, Specializing Gate Sets; the paper's U3 + CNOT
# evaluation set, Sec. V).  Every gate is stored as a 4 x 4 matrix on its two
# locations; single-qubit kinds act on loc[0] and are stored as g (x) I_2
# (loc[1] is only a partner qubit for the embedding).  With
# E2 = Tr over the partner of E (E2[a, b] = sum_c E[2a + c, 2b + c]),
# Re Tr(E (g (x) I)) = Re Tr(E2 g), so each single-qubit update maximises
# Re Tr(M2 g) with M2 = (1 - beta) E2 + beta g_old^dagger.
#   KIND_U4    general U(4): the SVD update above
#   KIND_FIXED applied but never optimised (e.g. CNOT)
#   KIND_U2    general U(2): SVD of M2 (maximiser Y X^dagger)
#   KIND_RZ    Rz(t) = diag(1, e^{it}): Re Tr(M2 Rz) = Re M2[0,0] +
#              |M2[1,1]| cos(t + arg M2[1,1]), maximal at t = -arg M2[1,1]
#   KIND_GPI   GPI(f) = [[0, e^{-if}], [e^{if}, 0]]: Re Tr(M2 GPI) =
#              Re((M2[0,1] + conj(M2[1,0])) e^{if}), maximal at
#              f = -arg(M2[0,1] + conj(M2[1,0]))
#   KIND_MS    the two-qubit Molmer-Sorensen gate MS(f1, f2) (both qubits):
#              with s = f1 + f2 and d = f1 - f2, Re Tr(M MS) is a constant
#              plus Re(w_s e^{is}) + Re(w_d e^{id}) (over sqrt 2), where
#              w_s = -i M[0,3] + i conj(M[3,0]) and w_d = -i M[1,2] +
#              i conj(M[2,1]), M = (1 - beta) E + beta u_old^dagger; s and d
#              are independent, so e^{is} = conj(w_s)/|w_s|, e^{id} likewise.
# A zero quantity to take the argument of (modulus below 1e-300) keeps the
# old gate, like a zero environment (Q15).
# ---------------------------------------------------------------------------

KIND_U4, KIND_FIXED, KIND_U2, KIND_RZ, KIND_GPI, KIND_MS = 0, 1, 2, 3, 4, 5


def rz(t: float) -> np.ndarray:
    return np.array([[1.0, 0.0], [0.0, np.exp(1j * t)]], np.complex128)


def gpi(f: float) -> np.ndarray:
    return np.array([[0.0, np.exp(-1j * f)], [np.exp(1j * f), 0.0]], np.complex128)


def ms(f1: float, f2: float) -> np.ndarray:
    """MS(f1, f2) = exp(-i pi/4 sigma_f1 (x) sigma_f2), sigma_f = cos f X + sin f Y."""
    es, ed = np.exp(1j * (f1 + f2)), np.exp(1j * (f1 - f2))
    return np.array([[1, 0, 0, -1j / es], [0, 1, -1j / ed, 0], [0, -1j * ed, 1, 0], [-1j * es, 0, 0, 1]],
                    np.complex128) / np.sqrt(2.0)


def _ms_from_phases(us: complex, ud: complex) -> np.ndarray:
    return np.array([[1, 0, 0, -1j * np.conj(us)], [0, 1, -1j * np.conj(ud), 0], [0, -1j * ud, 1, 0],
                     [-1j * us, 0, 0, 1]], np.complex128) / np.sqrt(2.0)


def _partner_trace(E: np.ndarray) -> np.ndarray:
    return np.einsum("acbc->ab", E.reshape(2, 2, 2, 2))


def optimize_gate_kind(E: np.ndarray, u_old: np.ndarray, kind: int, beta: float = 0.0) -> np.ndarray:
    """Gate update for every kind (see the table above); returns the 4 x 4
    stored matrix."""
    if kind == KIND_U4:
        return optimize_gate(E, u_old, beta)
    if kind == KIND_FIXED:
        return u_old.copy()
    if kind == KIND_MS:
        M = (1.0 - beta) * E + beta * u_old.conj().T
        if not np.all(np.isfinite(M)):
            return np.full_like(u_old, np.nan)
        ws = -1j * M[0, 3] + 1j * np.conj(M[3, 0])
        wd = -1j * M[1, 2] + 1j * np.conj(M[2, 1])
        if abs(ws) < 1e-300 or abs(wd) < 1e-300:
            return u_old.copy()
        return _ms_from_phases(np.conj(ws) / abs(ws), np.conj(wd) / abs(wd))
    g_old = u_old[::2, ::2]  # g of g (x) I_2
    M = (1.0 - beta) * _partner_trace(E) + beta * g_old.conj().T
    if not np.all(np.isfinite(M)):
        return np.full_like(u_old, np.nan)
    if kind == KIND_U2:
        scale = np.max(np.abs(M))
        if scale < 1e-300:
            return u_old.copy()
        Xs, _, Yh = np.linalg.svd(M / scale)
        g = Yh.conj().T @ Xs.conj().T
    elif kind == KIND_RZ:
        if abs(M[1, 1]) < 1e-300:
            return u_old.copy()
        g = rz(-np.angle(M[1, 1]))
    elif kind == KIND_GPI:
        w = M[0, 1] + np.conj(M[1, 0])
        if abs(w) < 1e-300:
            return u_old.copy()
        g = gpi(-np.angle(w))
    else:
        raise ValueError(kind)
    return np.kron(g, np.eye(2))


def optimize_gate_batched(E: np.ndarray, u_old: np.ndarray, beta: float = 0.0) -> np.ndarray:
    """optimize_gate over a leading batch axis (one stacked LAPACK SVD call;
    the zero and non-finite guards are applied per entry afterwards)."""
    M = (1.0 - beta) * E + beta * np.conj(np.swapaxes(u_old, -1, -2))
    finite = np.all(np.isfinite(M), axis=(-2, -1))
    scale = np.max(np.abs(np.where(finite[:, None, None], M, 0.0)), axis=(-2, -1))
    zero = scale < 1e-300
    Ms = np.where((finite & ~zero)[:, None, None], M / np.where(zero, 1.0, scale)[:, None, None], np.eye(M.shape[-1]))
    Xs, _, Yh = np.linalg.svd(Ms)
    out = np.conj(np.swapaxes(Yh, -1, -2)) @ np.conj(np.swapaxes(Xs, -1, -2))
    out = np.where(zero[:, None, None], u_old, out)
    return np.where(finite[:, None, None], out, np.nan + 0j)


# ---------------------------------------------------------------------------
# Definition mode: every environment from scratch (Alg. 1 order, Q5).
# ---------------------------------------------------------------------------

def sweep_definition(V, gates, locs, n: int, beta: float = 0.0, record: list | None = None, kinds=None):
    """One TwoSidedSweep with environments recomputed from scratch.  Returns
    the new gate list; if `record` is a list, appends (g, half, E, u_new, T)
    per update, T being Tr(V^dagger C) after the update."""
    gates = [np.array(u, dtype=np.complex128) for u in gates]
    p = len(gates)
    order = [(g, 0) for g in range(p - 1, -1, -1)] + [(g, 1) for g in range(p)]
    for g, half in order:
        E = environment(V, gates, locs, n, g)
        k = KIND_U4 if kinds is None else int(kinds[g])
        gates[g] = optimize_gate_kind(E, gates[g], k, beta)
        if record is not None:
            record.append((g, half, E, gates[g].copy(), complex(np.trace(E @ gates[g]))))
    return np.stack(gates)


# ---------------------------------------------------------------------------
# Builder mode: the circuit tensor of Alg. 1 (Q3, Q4), batched over starts.
# ---------------------------------------------------------------------------

class BuilderOracle:
    """Alg. 1 with the circuit tensor kept as an S x N x N complex128 array.

    InitCircuitTensor: X = V^dagger, then X <- G_g X for g = 1..p.
    First half (g = p..1): X <- G_g^dagger X, E = Tr_rest X, update,
    X <- X G_g'.  Second half (g = 1..p): X <- X G_g'^dagger, E = Tr_rest X,
    update, X <- G_g'' X."""

    def __init__(self, V: np.ndarray, gates: np.ndarray, locs, n: int, beta: float = 0.0, kinds=None):
        self.kinds = None if kinds is None else [int(k) for k in kinds]
        self.V = np.asarray(V, np.complex128)
        self.n = n
        self.N = 1 << n
        self.locs = [tuple(int(q) for q in l) for l in locs]
        self.gates = np.array(gates, dtype=np.complex128)  # (S, p, 2^k, 2^k)
        if self.gates.ndim == 3:
            self.gates = self.gates[None]
        self.S = self.gates.shape[0]
        self.beta = beta
        self.rebuild()

    def rebuild(self):
        X = np.broadcast_to(self.V.conj().T, (self.S, self.N, self.N)).copy()
        for g, loc in enumerate(self.locs):
            X = apply_left(X, self.gates[:, g], loc, self.n)
        self.X = X

    def trace(self) -> np.ndarray:
        return np.trace(self.X, axis1=1, axis2=2)

    def costs(self) -> np.ndarray:
        return 1.0 - np.abs(self.trace()) / self.N

    def update(self, g: int, half: int, record: list | None = None, active=None):
        loc = self.locs[g]
        u = self.gates[:, g]
        ud = np.conj(np.swapaxes(u, -1, -2))
        if half == 0:
            self.X = apply_left(self.X, ud, loc, self.n)
        else:
            self.X = apply_right(self.X, ud, loc, self.n)
        E = partial_trace(self.X, loc, self.n)
        kind = KIND_U4 if self.kinds is None else self.kinds[g]
        if kind == KIND_U4:
            unew = optimize_gate_batched(E, u, self.beta)
        else:
            unew = np.stack([optimize_gate_kind(E[s], u[s], kind, self.beta) for s in range(self.S)])
        if active is not None:
            unew = np.where(active[:, None, None], unew, u)
        self.gates[:, g] = unew
        if half == 0:
            self.X = apply_right(self.X, unew, loc, self.n)
        else:
            self.X = apply_left(self.X, unew, loc, self.n)
        if record is not None:
            record.append((g, half, E.copy(), unew.copy(), self.trace().copy()))

    def sweep(self, record: list | None = None, active=None):
        p = len(self.locs)
        for g in range(p - 1, -1, -1):
            self.update(g, 0, record, active)
        for g in range(p):
            self.update(g, 1, record, active)


# ---------------------------------------------------------------------------
# Termination and multistart (Sec. III-A-2, Sec. IV-A; Q7-Q13).
# ---------------------------------------------------------------------------

@dataclass
class Options:
    """Hyperparameters with the defaults the paper recommends (Sec. III-A-2)."""

    dist_tol: float = 1e-10
    diff_tol_a: float = 0.0
    diff_tol_r: float = 1e-5
    long_diff_count: int = 100
    long_diff_r: float = 0.1
    min_iter: int = 0
    max_iter: int = 100000
    reset_iter: int = 40
    beta: float = 0.0


@dataclass
class Result:
    gates: np.ndarray          # (p, 2^k, 2^k) best start
    all_gates: np.ndarray      # (S, p, 2^k, 2^k)
    costs: np.ndarray          # (S,) final costs recomputed from scratch
    best_start: int
    sweeps: int
    status: int
    history: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))  # (sweeps+1, S)


def _plateau_flags(hist: list, i: int, opt: Options) -> np.ndarray:
    c_i = hist[i]
    flags = np.zeros_like(c_i, dtype=bool)
    if opt.diff_tol_a > 0.0 or opt.diff_tol_r > 0.0:
        flags |= (hist[i - 1] - c_i) <= (opt.diff_tol_a + opt.diff_tol_r * c_i)
    L = opt.long_diff_count
    if L > 0 and i >= L:
        flags |= (hist[i - L] - c_i) < (opt.long_diff_r * hist[i - L])
    return flags


def instantiate(V: np.ndarray, init_gates: np.ndarray, locs, n: int, tol: float | None = None,
                opt: Options | None = None, mode: str = "builder", kinds=None) -> Result:
    """Multistart QFactor in lockstep.  mode='builder' runs Alg. 1's circuit
    tensor (with resets); mode='definition' recomputes every environment."""
    opt = opt or Options()
    tol = opt.dist_tol if tol is None else tol
    init_gates = np.asarray(init_gates, np.complex128)
    if init_gates.ndim == 3:
        init_gates = init_gates[None]
    S, p = init_gates.shape[:2]
    N = 1 << n
    locs = [tuple(int(q) for q in l) for l in locs]

    if mode == "builder":
        b = BuilderOracle(V, init_gates, locs, n, opt.beta, kinds)
        cur = lambda: b.costs()  # noqa: E731
        gates_of = lambda: b.gates  # noqa: E731
    elif mode == "definition":
        G = init_gates.copy()
        cur = lambda: np.array([cost(V, G[s], locs, n) for s in range(S)])  # noqa: E731
        gates_of = lambda: G  # noqa: E731
    else:
        raise ValueError(mode)

    def clean(c):
        return np.where(np.isfinite(c), c, np.inf)

    hist = [clean(cur())]
    numeric = ~np.isfinite(hist[0])
    plateaued = numeric.copy()
    status = STATUS_MAX_ITER
    i = 0
    while i < opt.max_iter:
        i += 1
        active = ~numeric
        if mode == "builder":
            b.sweep(active=active)
            if opt.reset_iter > 0 and i % opt.reset_iter == 0:
                b.rebuild()
        else:
            for s in range(S):
                if active[s]:
                    G[s] = sweep_definition(V, G[s], locs, n, opt.beta, kinds=kinds)
        c = cur()
        bad = ~np.isfinite(c)
        numeric |= bad
        hist.append(np.where(numeric, np.inf, c))
        if i >= opt.min_iter:
            ci = hist[i]
            if np.any((ci < tol) & ~numeric):
                status = STATUS_CONVERGED
                break
            plateaued |= numeric | _plateau_flags(hist, i, opt)
            if np.all(plateaued):
                status = STATUS_PLATEAU
                break
    all_g = np.array(gates_of())
    final = np.array([cost(V, all_g[s], locs, n) if not numeric[s] else np.inf for s in range(S)])
    final = np.where(np.isfinite(final), final, np.inf)
    best = int(np.argmin(final))
    if np.all(numeric):
        status = STATUS_NUMERIC
    elif final[best] < tol:
        status = STATUS_CONVERGED
    return Result(all_g[best].copy(), all_g, final, best, i, status, np.array(hist))


def nuclear_norm(E: np.ndarray) -> float:
    return float(np.sum(np.linalg.svd(E, compute_uv=False)))


def frobenius_distance_sq(V: np.ndarray, C: np.ndarray) -> float:
    return float(np.sum(np.abs(C - V) ** 2))


# ---------------------------------------------------------------------------
# Gradient of the cost (Sec. II: the cost Delta, and the gradient-based
# optimisers of "Numerical Optimization in Instantiation"; Q6 environment).
# ---------------------------------------------------------------------------

def cost_gradient(V: np.ndarray, gates, locs, n: int) -> tuple[float, np.ndarray]:
    """Delta and, for every gate matrix u_g, the real gradient packed as a
    complex matrix: G_g[i, j] = dDelta/dRe u_g[i, j] + 1j dDelta/dIm u_g[i, j].

    With T = Tr(V^dagger C) = Tr(E_g u_g) (Q6), dT/du_g[i, j] = E_g[j, i], so
    d|T| along a change du is Re(conj(T) Tr(E_g du)) / |T|, which gives
    G_g = -(T / |T|) conj(E_g)^T / N.  At T = 0 the modulus is not
    differentiable; the zero matrix is returned there."""
    gates = np.asarray(gates, np.complex128)
    N = 1 << n
    T = overlap(V, circuit_unitary(gates, locs, n))
    G = np.zeros_like(gates)
    if abs(T) > 0.0:
        ph = T / abs(T)
        for g in range(len(gates)):
            E = environment(V, gates, locs, n, g)
            G[g] = -(ph / N) * E.conj().T
    return 1.0 - abs(T) / N, G


# Parameterised two-qubit gates for the gradient-based baseline: a gate is
# exp(i H(theta)) with H = sum_k theta_k P_k over the 15 non-identity
# two-qubit Pauli products P_k = sigma_a (x) sigma_b, (a, b) != (0, 0), in
# the order a = 0..3 major, b = 0..3 minor.  H is Hermitian and traceless, so
# the gate is in SU(4); the cost does not see a gate's global phase, so 15
# real parameters reach every U(4) gate up to that phase.

_SIGMA = [np.eye(2, dtype=np.complex128),
          np.array([[0, 1], [1, 0]], np.complex128),
          np.array([[0, -1j], [1j, 0]], np.complex128),
          np.array([[1, 0], [0, -1]], np.complex128)]
PAULI2 = np.stack([np.kron(_SIGMA[a], _SIGMA[b]) for a in range(4) for b in range(4) if (a, b) != (0, 0)])


def su4_hermitian(theta: np.ndarray) -> np.ndarray:
    """H(theta) = sum_k theta_k P_k for theta of shape (..., 15)."""
    return np.tensordot(np.asarray(theta, np.float64), PAULI2, axes=([-1], [0]))


def su4_gate(theta: np.ndarray) -> np.ndarray:
    """exp(i H(theta)) for theta of shape (..., 15) (matrix exponential)."""
    from scipy.linalg import expm
    th = np.asarray(theta, np.float64)
    flat = th.reshape(-1, 15)
    out = np.stack([expm(1j * su4_hermitian(t)) for t in flat])
    return out.reshape(th.shape[:-1] + (4, 4))


def su4_theta_gradient(theta: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Chain rule from a gate-matrix gradient G (packed as in cost_gradient)
    to the 15 parameters: dDelta/dtheta_k = Re Tr(G^dagger dU/dtheta_k), with
    dU/dtheta_k the Frechet derivative of the exponential at iH in the
    direction iP_k."""
    from scipy.linalg import expm_frechet
    th = np.asarray(theta, np.float64).reshape(-1, 15)
    Gf = np.asarray(G, np.complex128).reshape(-1, 4, 4)
    out = np.zeros_like(th)
    for i in range(th.shape[0]):
        A = 1j * su4_hermitian(th[i])
        for k in range(15):
            dU = expm_frechet(A, 1j * PAULI2[k], compute_expm=False)
            out[i, k] = float(np.real(np.vdot(Gf[i], dU)))
    return out.reshape(np.shape(theta))


def param_cost_gradient(V: np.ndarray, theta: np.ndarray, locs, n: int) -> tuple[float, np.ndarray]:
    """Delta and dDelta/dtheta for gates exp(i H(theta_g)), theta (p, 15)."""
    gates = su4_gate(theta)
    c, G = cost_gradient(V, gates, locs, n)
    return c, su4_theta_gradient(theta, G)
