"""Pins of the phonon self-energy oracle (Eqs. (4)-(5)), of the D~ combination
and of the retarded relation against facts fixed by the paper and by
mathematics: a 2-D FFT correlation (periodic in kz, zero-padded in E), the
single-term reduction to a trace of four matrices, a closed form for
constant G, a worked example, the (anti-)Hermitian symmetry the equations
imply, exact equivariances, bilinearity, the diagonal's relation to the
neighbour blocks, and the sampled evaluation against the full one.  Each pin
returns the worst error it saw (0 for exact pins) and raises AssertionError
on failure.
"""
from __future__ import annotations

import numpy as np

import oracle
from tests.pins import _ratio, _rel, rand_antiherm


def pi_problem(rng, NA=6, NB=3, Norb=3, Nkz=3, Nqz=2, NE=9, shift=(1, 2, 4), neigh=None):
    shift = np.asarray(shift, dtype=np.int32)
    if neigh is None:
        neigh = np.stack([rng.choice([x for x in range(NA) if x != a], NB, replace=False)
                          for a in range(NA)]).astype(np.int32)
    dH = rng.standard_normal((NA, NB, 3, Norb, Norb))
    X = rand_antiherm(rng, (Nkz, NE, NA, Norb, Norb))
    Y = rand_antiherm(rng, (Nkz, NE, NA, Norb, Norb))
    return dict(neigh=neigh, dH=dH, X=X, Y=Y, shift=shift, Nkz=Nkz, Nqz=Nqz, NE=NE)


def pin_pi_single_term(lib=oracle.PI_LIB):
    """Nkz = Nqz = NE = Nw = 1 with s = 0: each neighbour block is
    beta tr(dH_ab,i^T X_a dH_ab,j Y_f), a trace of a product of four matrices
    (numpy matmul), and the diagonal is -beta times their sum over b."""
    rng = np.random.default_rng(31)
    NA, NB, Norb = 4, 2, 3
    neigh = np.array([[2, 1], [0, 3], [3, 0], [1, 2]], dtype=np.int32)
    dH = rng.standard_normal((NA, NB, 3, Norb, Norb))
    X = rng.standard_normal((1, 1, NA, Norb, Norb)) + 1j * rng.standard_normal((1, 1, NA, Norb, Norb))
    Y = rng.standard_normal((1, 1, NA, Norb, Norb)) + 1j * rng.standard_normal((1, 1, NA, Norb, Norb))
    beta = 0.4 + 1.3j
    got = oracle.pi(neigh, dH, X, Y, [0], 1, 1, 1, beta=beta, lib=lib)
    want = np.zeros_like(got)
    for a in range(NA):
        for b in range(NB):
            f = neigh[a, b]
            for i in range(3):
                for j in range(3):
                    m = dH[a, b, i].T @ X[0, 0, a] @ dH[a, b, j] @ Y[0, 0, f]
                    want[0, 0, a, b, i, j] = beta * np.trace(m)
        want[0, 0, a, NB] = -want[0, 0, a, :NB].sum(axis=0)
    err = _rel(got, want)
    assert err < 1e-14, err
    return err


def pin_pi_fft_correlation(lib=oracle.PI_LIB):
    """Norb = NA = NB = 1 (the atom its own neighbour), dH = 1: Eq. (5) is the
    2-D cross-correlation P[q, s] = sum_k sum_e X[k + q, e + s] Y[k, e],
    periodic in kz and zero-padded in E, evaluated here by FFT."""
    rng = np.random.default_rng(32)
    Nkz, Nqz, NE = 5, 4, 13
    shift = np.array([1, 3, -2, 5, 0], dtype=np.int32)
    neigh = np.zeros((1, 1), dtype=np.int32)
    dH = np.ones((1, 1, 3, 1, 1))
    X = rng.standard_normal((Nkz, NE)) + 1j * rng.standard_normal((Nkz, NE))
    Y = rng.standard_normal((Nkz, NE)) + 1j * rng.standard_normal((Nkz, NE))
    got = oracle.pi(neigh, dH, X.reshape(Nkz, NE, 1, 1, 1), Y.reshape(Nkz, NE, 1, 1, 1), shift,
                    Nkz, Nqz, NE, beta=1j, lib=lib)
    L = 2 * NE + 2 * int(np.abs(shift).max())
    x = np.zeros((Nkz, L), dtype=np.complex128)
    x[:, :NE] = X
    yr = np.zeros((Nkz, L), dtype=np.complex128)       # y reversed in both axes
    yr[:, :NE] = Y
    yr = np.roll(yr[::-1, ::-1], 1, axis=(0, 1))
    c = np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(yr))  # c[q, s] = sum x[k+q, e+s] y[k, e]
    want_off = 1j * np.stack([c[:Nqz, s % L] for s in shift], axis=1)
    err = 0.0
    for i in range(3):
        for j in range(3):
            err = max(err, _rel(got[:, :, 0, 0, i, j], want_off))
            err = max(err, _rel(got[:, :, 0, 1, i, j], -want_off))
    assert err < 1e-13, err
    return err


def pin_pi_closed_form_constant(lib=oracle.PI_LIB):
    """X_a and Y_f constant over (kz, E): the sums collapse to
    Nkz * n(s_w) * tr(dH_i^T X_a dH_j Y_f), n(s) = #{e : 0 <= e + s < NE}."""
    rng = np.random.default_rng(33)
    NA, NB, Norb, Nkz, Nqz, NE = 5, 2, 3, 3, 2, 8
    shift = np.array([1, -3, 6, 0], dtype=np.int32)
    neigh = np.array([[1, 2], [3, 4], [0, 4], [2, 1], [3, 0]], dtype=np.int32)
    dH = rng.standard_normal((NA, NB, 3, Norb, Norb))
    Xc = rand_antiherm(rng, (NA, Norb, Norb))
    Yc = rand_antiherm(rng, (NA, Norb, Norb))
    X = np.broadcast_to(Xc, (Nkz, NE, NA, Norb, Norb)).copy()
    Y = np.broadcast_to(Yc, (Nkz, NE, NA, Norb, Norb)).copy()
    got = oracle.pi(neigh, dH, X, Y, shift, Nkz, Nqz, NE, beta=1j, lib=lib)
    n_s = np.array([np.sum((np.arange(NE) + s >= 0) & (np.arange(NE) + s < NE)) for s in shift])
    want = np.zeros_like(got)
    for a in range(NA):
        for b in range(NB):
            for i in range(3):
                for j in range(3):
                    t = np.trace(dH[a, b, i].T @ Xc[a] @ dH[a, b, j] @ Yc[neigh[a, b]])
                    want[:, :, a, b, i, j] = 1j * Nkz * n_s[None, :] * t
        want[:, :, a, NB] = -want[:, :, a, :NB].sum(axis=2)
    err = _rel(got, want)
    assert err < 1e-13, err
    return err


def pin_pi_hand_example(lib=oracle.PI_LIB):
    """A worked example small enough to do by hand: Norb = 2, one atom that is
    its own neighbour, Nkz = Nqz = 1, one frequency (s = 1), NE = 2,
    dH_x = [[1, 2], [0, 1]], dH_y = dH_z = 0, X(E=1) = [[i, 1], [-1, 2i]],
    Y(E=0) = [[2, 1], [i, 0]].  dH_x^T X = [[i, 1], [2i-1, 2+2i]];
    (dH_x^T X) dH_x = [[i, 1+2i], [2i-1, 6i]];  trace with Y:
    2i + (1+2i) i + (2i-1) + 0 = -3+5i.  Pi_ab,xx = i(-3+5i) = -5-3i,
    Pi_aa,xx = 5+3i, every other entry 0."""
    neigh = np.zeros((1, 1), dtype=np.int32)
    dH = np.zeros((1, 1, 3, 2, 2))
    dH[0, 0, 0] = [[1, 2], [0, 1]]
    X = np.zeros((1, 2, 1, 2, 2), dtype=np.complex128)
    Y = np.zeros((1, 2, 1, 2, 2), dtype=np.complex128)
    X[0, 1, 0] = [[1j, 1], [-1, 2j]]
    X[0, 0, 0] = [[7, 7], [7, 7]]   # never read: E + s = 0 needs E = -1
    Y[0, 0, 0] = [[2, 1], [1j, 0]]
    Y[0, 1, 0] = [[9, 9], [9, 9]]   # never read: E = 1 needs X(E=2), outside the grid
    got = oracle.pi(neigh, dH, X, Y, [1], 1, 1, 2, beta=1j, lib=lib)
    want = np.zeros((1, 1, 1, 2, 3, 3), dtype=np.complex128)
    want[0, 0, 0, 0, 0, 0] = -5 - 3j
    want[0, 0, 0, 1, 0, 0] = 5 + 3j
    assert np.array_equal(got, want), got
    return 0.0


def pin_pi_antihermitian(lib=oracle.PI_LIB):
    """For anti-Hermitian G< and G> and real dH the trace of Eq. (5) satisfies
    conj(P_ij) = P_ji, so with beta = i every 3 x 3 block of Pi (neighbour and
    diagonal) is anti-Hermitian -- the symmetry of a lesser/greater
    self-energy -- and with beta = 1 Hermitian."""
    rng = np.random.default_rng(34)
    p = pi_problem(rng)
    p_i = oracle.pi(beta=1j, lib=lib, **p)
    p_1 = oracle.pi(beta=1.0, lib=lib, **p)
    sh = lambda x: np.conj(np.swapaxes(x, -1, -2))
    e1 = _ratio(p_i + sh(p_i), p_i)
    e2 = _ratio(p_1 - sh(p_1), p_1)
    assert e1 < 1e-14 and e2 < 1e-14, (e1, e2)
    assert np.linalg.norm(p_i) > 1.0
    return max(e1, e2)


def pin_pi_kz_roll(lib=oracle.PI_LIB):
    """With Nqz = Nkz, rolling X by one kz point rolls Pi by one qz point,
    exactly; rolling Y by one point rolls it the other way (kz periodic)."""
    rng = np.random.default_rng(35)
    p = pi_problem(rng, Nkz=4, Nqz=4)
    p0 = oracle.pi(lib=lib, **p)
    px = oracle.pi(lib=lib, **dict(p, X=np.roll(p["X"], 1, axis=0)))
    assert np.array_equal(px, np.roll(p0, 1, axis=0))
    py = oracle.pi(lib=lib, **dict(p, Y=np.roll(p["Y"], 1, axis=0)))
    err = _rel(py, np.roll(p0, -1, axis=0))
    assert err < 1e-14, err
    return err


def pin_pi_energy_shift_and_edge(lib=oracle.PI_LIB):
    """Shifting X up one energy point (its top row zero beforehand) acts as
    shift s_w - 1; a shift of NE - 1 keeps only the term e = 0; a shift of
    -(NE - 1) only e = NE - 1."""
    rng = np.random.default_rng(36)
    NE = 10
    p = pi_problem(rng, NE=NE, shift=(2, 3, 5, 0))
    X0 = p["X"].copy()
    X0[:, NE - 1] = 0
    X1 = np.zeros_like(X0)
    X1[:, 1:] = X0[:, :-1]
    base = dict(p, X=X0)
    lower = oracle.pi(lib=lib, **dict(base, shift=np.array([1, 2, 4, -1], dtype=np.int32)))
    up = oracle.pi(lib=lib, **dict(base, X=X1))
    err = _rel(up, lower)
    assert err < 1e-15, err
    # extreme shifts: one energy term each
    one = dict(p, shift=np.array([NE - 1, -(NE - 1)], dtype=np.int32))
    got = oracle.pi(lib=lib, **one)
    Xe = np.zeros_like(p["X"])
    Ye = np.zeros_like(p["Y"])
    Xe[:, NE - 1] = p["X"][:, NE - 1]
    Ye[:, 0] = p["Y"][:, 0]
    want_hi = oracle.pi(lib=lib, **dict(one, X=Xe, Y=Ye))[:, 0]
    Xe = np.zeros_like(p["X"])
    Ye = np.zeros_like(p["Y"])
    Xe[:, 0] = p["X"][:, 0]
    Ye[:, NE - 1] = p["Y"][:, NE - 1]
    want_lo = oracle.pi(lib=lib, **dict(one, X=Xe, Y=Ye))[:, 1]
    e2 = max(_rel(got[:, 0], want_hi), _rel(got[:, 1], want_lo))
    assert e2 < 1e-15, e2
    assert np.linalg.norm(got[:, 0]) > 0 and np.linalg.norm(got[:, 1]) > 0
    return max(err, e2)


def pin_pi_bilinear(lib=oracle.PI_LIB):
    """Pi is linear in X and in Y (complex coefficients)."""
    rng = np.random.default_rng(37)
    p = pi_problem(rng)
    q = pi_problem(np.random.default_rng(38))
    c1, c2 = 0.7 - 0.2j, -1.3 + 0.4j
    sX = oracle.pi(lib=lib, **dict(p, X=c1 * p["X"] + c2 * q["X"]))
    wX = c1 * oracle.pi(lib=lib, **p) + c2 * oracle.pi(lib=lib, **dict(p, X=q["X"]))
    sY = oracle.pi(lib=lib, **dict(p, Y=c1 * p["Y"] + c2 * q["Y"]))
    wY = c1 * oracle.pi(lib=lib, **p) + c2 * oracle.pi(lib=lib, **dict(p, Y=q["Y"]))
    e = max(_rel(sX, wX), _rel(sY, wY))
    assert e < 1e-13, e
    return e


def pin_pi_diagonal(lib=oracle.PI_LIB):
    """The diagonal block (Eq. (4), -i sum over the neighbours) is minus the sum
    of the neighbour blocks (Eq. (5), +i)."""
    rng = np.random.default_rng(39)
    p = pi_problem(rng, NB=4, NA=7)
    got = oracle.pi(lib=lib, **p)
    NB = p["neigh"].shape[1]
    err = _rel(got[:, :, :, NB], -got[:, :, :, :NB].sum(axis=3))
    assert err < 1e-14, err
    return err


def pin_pi_atom_relabel(lib=oracle.PI_LIB):
    """Relabelling atoms permutes Pi the same way, exactly."""
    rng = np.random.default_rng(40)
    p = pi_problem(rng)
    NA = p["dH"].shape[0]
    perm = rng.permutation(NA)
    inv = np.argsort(perm)
    p1 = dict(p, X=p["X"][:, :, inv], Y=p["Y"][:, :, inv],
              neigh=perm[p["neigh"][inv]].astype(np.int32), dH=p["dH"][inv])
    assert np.array_equal(oracle.pi(lib=lib, **p1), oracle.pi(lib=lib, **p)[:, :, inv])
    return 0.0


def _pi_sampled_case():
    rng = np.random.default_rng(41)
    p = pi_problem(rng, NA=7, NB=3, Norb=3, Nkz=4, Nqz=3, NE=12, shift=(3, -2, 1, 11))
    blocks = [(0, 0, 0), (2, 3, 6), (1, 1, 2), (0, 2, 6), (2, 0, 0), (1, 3, 3), (0, 0, 0),
              (2, 1, 5)]
    return p, np.array(blocks, dtype=np.int32)


def pin_pi_sampled_blocks(lib=oracle.PI_LIB):
    """The sampled evaluation (listed (q, w, a) blocks; G as stacks of only the
    blocks they read, located through gslot) reproduces the full evaluation
    bit for bit, and withholding any listed G block is reported as missing."""
    p, blocks = _pi_sampled_case()
    Nkz, NE = p["Nkz"], p["NE"]
    NA, Norb = p["dH"].shape[0], p["dH"].shape[3]
    full = oracle.pi(lib=lib, **p)
    want = full[blocks[:, 0], blocks[:, 1], blocks[:, 2]]
    got = oracle.pi(lib=lib, blocks=blocks, **p)
    assert np.array_equal(got, want)
    need = oracle.needed_g_blocks_pi(p["neigh"], p["shift"], Nkz, NE, NA, blocks)
    order = np.random.default_rng(42).permutation(need.size)
    gslot = np.full(Nkz * NE * NA, -1, dtype=np.int64)
    gslot[need[order]] = np.arange(need.size)
    Xs = p["X"].reshape(-1, Norb, Norb)[need[order]]
    Ys = p["Y"].reshape(-1, Norb, Norb)[need[order]]
    got2 = oracle.pi(lib=lib, blocks=blocks, gslot=gslot, **dict(p, X=Xs, Y=Ys))
    assert np.array_equal(got2, want)
    for drop in range(0, need.size, 7):
        keep = np.delete(need, drop)
        gs = np.full(Nkz * NE * NA, -1, dtype=np.int64)
        gs[keep] = np.arange(keep.size)
        try:
            oracle.pi(lib=lib, blocks=blocks, gslot=gs,
                      **dict(p, X=p["X"].reshape(-1, Norb, Norb)[keep],
                             Y=p["Y"].reshape(-1, Norb, Norb)[keep]))
        except ValueError:
            continue
        raise AssertionError(f"block {need[drop]} withheld but not reported missing")
    return 0.0


def sym_neigh(rng, NA, NB):
    """A symmetric neighbour table: atoms on a ring in a random order, each
    joined to the NB/2 nearest on either side (NB even, NA > NB)."""
    order = rng.permutation(NA)
    pos = np.argsort(order)
    offs = [o for d in range(1, NB // 2 + 1) for o in (d, -d)]
    return np.array([[order[(pos[a] + o) % NA] for o in offs] for a in range(NA)],
                    dtype=np.int32)


def pin_dtilde_structure():
    """D~ of Eq. (3): a D whose neighbour blocks are all equal to its diagonal
    blocks (D_ab = D_aa = D_bb = D_ba = C) gives D~ = 0; a D whose only nonzero
    blocks are the diagonal ones gives D~_ab = -(D_aa + D_bb); a D with one
    nonzero neighbour block D_a0,b0 gives D~ = that block at (a0, b0) and at
    the reverse pair (b0 -> a0), zero elsewhere."""
    rng = np.random.default_rng(43)
    NA, NB, Nqz, Nw = 9, 4, 2, 3
    neigh = sym_neigh(rng, NA, NB)
    shape = (Nqz, Nw, NA, NB + 1, 3, 3)
    C = rng.standard_normal((Nqz, Nw, 1, 1, 3, 3)) + 1j * rng.standard_normal((Nqz, Nw, 1, 1, 3, 3))
    assert np.array_equal(oracle.dtilde(np.broadcast_to(C, shape), neigh),
                          np.zeros((Nqz, Nw, NA, NB, 3, 3)))
    Dd = np.zeros(shape, dtype=np.complex128)
    Dd[:, :, :, NB] = rng.standard_normal((Nqz, Nw, NA, 3, 3))
    got = oracle.dtilde(Dd, neigh)
    want = -(Dd[:, :, :, NB][:, :, :, None] + Dd[:, :, neigh, NB])
    assert np.array_equal(got, want)
    D1 = np.zeros(shape, dtype=np.complex128)
    a0, b0 = 3, 2
    f0 = neigh[a0, b0]
    r0 = int(np.nonzero(neigh[f0] == a0)[0][0])
    D1[:, :, a0, b0] = C[:, :, 0, 0]
    got = oracle.dtilde(D1, neigh)
    want = np.zeros((Nqz, Nw, NA, NB, 3, 3), dtype=np.complex128)
    want[:, :, a0, b0] = C[:, :, 0, 0]
    want[:, :, f0, r0] = C[:, :, 0, 0]
    assert np.array_equal(got, want)
    # an asymmetric table is refused
    bad = neigh.copy()
    bad[0, 0] = [x for x in range(NA) if x not in neigh[0] and x != 0][0]
    try:
        oracle.dtilde(Dd, bad)
    except ValueError:
        return 0.0
    raise AssertionError("asymmetric neighbour table accepted")


def pin_dtilde_sigma_antihermitian():
    """Anti-Hermitian 3 x 3 blocks of D give an anti-Hermitian D~ (a sum of
    them), and so, through Eq. (3), an anti-Hermitian Sigma< (alpha = i)."""
    rng = np.random.default_rng(44)
    NA, NB, Nqz, Nw, Norb, Nkz, NE = 7, 2, 2, 3, 3, 3, 8
    neigh = sym_neigh(rng, NA, NB)
    D = rand_antiherm(rng, (Nqz, Nw, NA, NB + 1, 3, 3))
    Dt = oracle.dtilde(D, neigh)
    sh = lambda x: np.conj(np.swapaxes(x, -1, -2))
    e1 = _ratio(Dt + sh(Dt), Dt)
    dH = rng.standard_normal((NA, NB, 3, Norb, Norb))
    G = rand_antiherm(rng, (Nkz, NE, NA, Norb, Norb))
    S = oracle.sigma(neigh, dH, G, Dt, [1, 2, 3], Nkz, NE, alpha=1j)
    e2 = _ratio(S + sh(S), S)
    assert e1 == 0.0 and e2 < 1e-14, (e1, e2)
    return e2


def pin_retarded():
    """The retarded relation (X> - X<)/2: zero when the two components agree,
    X>/2 when the lesser one is zero, odd under exchanging them, and, for
    anti-Hermitian lesser/greater blocks, anti-Hermitian."""
    rng = np.random.default_rng(45)
    L = rand_antiherm(rng, (3, 4, 5, 5))
    Gt = rand_antiherm(rng, (3, 4, 5, 5))
    assert np.array_equal(oracle.retarded(L, L), np.zeros_like(L))
    assert np.array_equal(oracle.retarded(np.zeros_like(L), Gt), Gt / 2)
    assert np.array_equal(oracle.retarded(Gt, L), -oracle.retarded(L, Gt))
    R = oracle.retarded(L, Gt)
    e = _ratio(R + np.conj(np.swapaxes(R, -1, -2)), R)
    assert e == 0.0, e
    return e


PI_PINS = [pin_pi_single_term, pin_pi_fft_correlation, pin_pi_closed_form_constant,
           pin_pi_hand_example, pin_pi_antihermitian, pin_pi_kz_roll,
           pin_pi_energy_shift_and_edge, pin_pi_bilinear, pin_pi_diagonal, pin_pi_atom_relabel,
           pin_pi_sampled_blocks]
OTHER_PINS = [pin_dtilde_structure, pin_dtilde_sigma_antihermitian, pin_retarded]
