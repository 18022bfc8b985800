"""Pins of the oracle against facts fixed by the paper and by mathematics.

Each pin evaluates the oracle (optionally a rebuilt copy at ``lib``) and
compares it with something that does not restate Eq. (3)'s loop nest:
closed forms, a 2-D FFT correlation, plain matrix products of a single-term
reduction, exact equivariances and the (anti-)Hermitian symmetry that Eq. (3)
implies for anti-Hermitian G and D~.  Each returns the worst error it saw
(0 for exact pins) and raises AssertionError on failure.
"""
from __future__ import annotations

import numpy as np

import oracle
import ssegen

SEED = 1912


def rand_antiherm(rng, shape):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return 0.5 * (x - np.conj(np.swapaxes(x, -1, -2)))


def small_problem(rng, NA=6, NB=3, Norb=3, N3D=3, Nkz=3, Nqz=2, NE=9, shift=(1, 2, 4)):
    shift = np.asarray(shift, dtype=np.int32)
    Nw = shift.size
    neigh = np.stack([rng.choice([x for x in range(NA) if x != a], NB, replace=False)
                      for a in range(NA)]).astype(np.int32)
    dH = rng.standard_normal((NA, NB, N3D, Norb, Norb))
    G = rand_antiherm(rng, (Nkz, NE, NA, Norb, Norb))
    D = rand_antiherm(rng, (Nqz, Nw, NA, NB, N3D, N3D))
    return dict(neigh=neigh, dH=dH, G=G, D=D, shift=shift, Nkz=Nkz, NE=NE)


def _rel(x, y):
    """Relative Frobenius distance |x - y| / |y|."""
    return float(np.linalg.norm((x - y).ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


def _ratio(x, y):
    """|x| / |y| (Frobenius)."""
    return float(np.linalg.norm(x.ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


def pin_single_term(lib=oracle.LIB):
    """NB = Nqz = Nw = 1 and D~ nonzero at a single (i0, j0): Eq. (3) reduces to
    Sigma[k, e, a] = alpha D~ dH_i0 G_f(k, e - s) dH_j0^T, a product of three matrices."""
    rng = np.random.default_rng(11)
    worst = 0.0
    NA, Norb, Nkz, NE, s = 4, 3, 2, 6, 2
    neigh = np.array([[2], [0], [3], [1]], dtype=np.int32)
    dH = rng.standard_normal((NA, 1, 3, Norb, Norb))
    G = rng.standard_normal((Nkz, NE, NA, Norb, Norb)) + 1j * rng.standard_normal(
        (Nkz, NE, NA, Norb, Norb))
    for i0 in range(3):
        for j0 in range(3):
            D = np.zeros((1, 1, NA, 1, 3, 3), dtype=np.complex128)
            D[0, 0, :, 0, i0, j0] = rng.standard_normal(NA) + 1j * rng.standard_normal(NA)
            alpha = 0.3 - 1.7j
            got = oracle.sigma(neigh, dH, G, D, [s], Nkz, NE, alpha=alpha, lib=lib)
            want = np.zeros_like(got)
            for k in range(Nkz):
                for e in range(s, NE):
                    for a in range(NA):
                        f = neigh[a, 0]
                        want[k, e, a] = alpha * D[0, 0, a, 0, i0, j0] * (
                            dH[a, 0, i0] @ G[k, e - s, f] @ dH[a, 0, j0].T)
            err = _rel(got, want)
            assert err < 1e-14, (i0, j0, err)
            worst = max(worst, err)
    return worst


def pin_fft_correlation(lib=oracle.LIB):
    """Norb = NA = NB = 1, dH = 1, D~ only at (0, 0): Eq. (3) is a 2-D
    correlation, periodic in kz and zero-padded in E, evaluated here by FFT."""
    rng = np.random.default_rng(12)
    Nkz, Nqz, NE = 5, 3, 13
    shift = np.array([1, 3, -2, 5], dtype=np.int32)  # any integer shifts, both signs
    Nw = shift.size
    neigh = np.zeros((1, 1), dtype=np.int32)
    dH = np.ones((1, 1, 3, 1, 1))
    G = rng.standard_normal((Nkz, NE, 1, 1, 1)) + 1j * rng.standard_normal((Nkz, NE, 1, 1, 1))
    D = np.zeros((Nqz, Nw, 1, 1, 3, 3), dtype=np.complex128)
    D[:, :, 0, 0, 0, 0] = rng.standard_normal((Nqz, Nw)) + 1j * rng.standard_normal((Nqz, Nw))
    got = oracle.sigma(neigh, dH, G, D, shift, Nkz, NE, alpha=1j, lib=lib)[:, :, 0, 0, 0]
    L = NE + int(np.abs(shift).max()) + 1
    g = np.zeros((Nkz, L), dtype=np.complex128)
    g[:, :NE] = G[:, :, 0, 0, 0]
    h = np.zeros((Nkz, L), dtype=np.complex128)
    for q in range(Nqz):
        for w in range(Nw):
            h[q, shift[w] % L] += D[q, w, 0, 0, 0, 0]
    want = 1j * np.fft.ifft2(np.fft.fft2(g) * np.fft.fft2(h))[:, :NE]
    err = _rel(got, want)
    assert err < 1e-13, err
    return err


def pin_closed_form_constant(lib=oracle.LIB):
    """G_f constant over (kz, E), D~ constant over (qz, w): the sums over q and w
    collapse to Nqz * n(e), n(e) = #{w : 0 <= e - s_w < NE}."""
    rng = np.random.default_rng(13)
    NA, NB, Norb, Nkz, Nqz, NE = 5, 2, 3, 3, 3, 8
    shift = np.array([1, 2, 6], dtype=np.int32)
    neigh = np.array([[1, 2], [3, 4], [0, 4], [2, 1], [3, 0]], dtype=np.int32)
    dH = rng.standard_normal((NA, NB, 3, Norb, Norb))
    Gc = rand_antiherm(rng, (NA, Norb, Norb))
    Dc = rng.standard_normal((NA, NB, 3, 3)) + 1j * rng.standard_normal((NA, NB, 3, 3))
    G = np.broadcast_to(Gc, (Nkz, NE, NA, Norb, Norb)).copy()
    D = np.broadcast_to(Dc, (Nqz, shift.size, NA, NB, 3, 3)).copy()
    got = oracle.sigma(neigh, dH, G, D, shift, Nkz, NE, alpha=1j, lib=lib)
    base = np.zeros((NA, Norb, Norb), dtype=np.complex128)
    for a in range(NA):
        for b in range(NB):
            for i in range(3):
                for j in range(3):
                    base[a] += Dc[a, b, i, j] * (dH[a, b, i] @ Gc[neigh[a, b]] @ dH[a, b, j].T)
    n_e = np.array([np.sum((e - shift >= 0) & (e - shift < NE)) for e in range(NE)])
    want = 1j * Nqz * n_e[None, :, None, None, None] * base[None, None]
    want = np.broadcast_to(want, got.shape)
    err = _rel(got, want)
    assert err < 1e-13, err
    return err


def pin_antihermitian(lib=oracle.LIB):
    """For anti-Hermitian G and D~ and real dH, Eq. (3) with alpha = i gives an
    anti-Hermitian Sigma (the symmetry of a lesser/greater self-energy); with
    alpha = 1 it gives a Hermitian one."""
    rng = np.random.default_rng(14)
    p = small_problem(rng)
    s_i = oracle.sigma(alpha=1j, lib=lib, **p)
    s_1 = oracle.sigma(alpha=1.0, lib=lib, **p)
    sh = lambda x: np.conj(np.swapaxes(x, -1, -2))
    e1 = _ratio(s_i + sh(s_i), s_i)
    e2 = _ratio(s_1 - sh(s_1), s_1)
    assert e1 < 1e-14 and e2 < 1e-14, (e1, e2)
    assert np.linalg.norm(s_i) > 1.0
    return max(e1, e2)


def pin_kz_roll(lib=oracle.LIB):
    """Rolling G by one kz point rolls Sigma by one point, exactly (kz periodic)."""
    rng = np.random.default_rng(15)
    p = small_problem(rng, Nkz=4, Nqz=3)
    s0 = oracle.sigma(lib=lib, **p)
    p1 = dict(p, G=np.roll(p["G"], 1, axis=0))
    s1 = oracle.sigma(lib=lib, **p1)
    assert np.array_equal(s1, np.roll(s0, 1, axis=0))
    return 0.0


def pin_energy_shift_and_edge(lib=oracle.LIB):
    """Shifting G up one energy point (zero at the bottom) shifts Sigma up one
    point exactly; Sigma vanishes below the smallest shift (zero-padded edge)."""
    rng = np.random.default_rng(16)
    p = small_problem(rng, NE=11, shift=(2, 3, 5))
    s0 = oracle.sigma(lib=lib, **p)
    G1 = np.zeros_like(p["G"])
    G1[:, 1:] = p["G"][:, :-1]
    s1 = oracle.sigma(lib=lib, **dict(p, G=G1))
    assert np.array_equal(s1[:, 1:], s0[:, :-1])
    assert np.array_equal(s0[:, :2], np.zeros_like(s0[:, :2]))
    assert np.all(np.abs(s0[:, 2]).sum(axis=(-1, -2)) > 0)
    return 0.0


def pin_atom_relabel(lib=oracle.LIB):
    """Relabelling atoms permutes Sigma the same way, exactly."""
    rng = np.random.default_rng(17)
    p = small_problem(rng)
    NA = p["dH"].shape[0]
    perm = rng.permutation(NA)  # atom a -> perm[a]
    inv = np.argsort(perm)
    G1 = p["G"][:, :, inv]
    neigh1 = perm[p["neigh"][inv]].astype(np.int32)
    dH1 = p["dH"][inv]
    D1 = p["D"][:, :, inv]
    s0 = oracle.sigma(lib=lib, **p)
    s1 = oracle.sigma(lib=lib, **dict(p, G=G1, neigh=neigh1, dH=dH1, D=D1))
    assert np.array_equal(s1, s0[:, :, inv])
    return 0.0


def pin_linearity(lib=oracle.LIB):
    """Sigma is linear in D~ and in G (complex coefficients)."""
    rng = np.random.default_rng(18)
    p = small_problem(rng)
    q = small_problem(np.random.default_rng(19))
    c1, c2 = 0.7 - 0.2j, -1.3 + 0.4j
    sD = oracle.sigma(lib=lib, **dict(p, D=c1 * p["D"] + c2 * q["D"]))
    wD = c1 * oracle.sigma(lib=lib, **p) + c2 * oracle.sigma(lib=lib, **dict(p, D=q["D"]))
    sG = oracle.sigma(lib=lib, **dict(p, G=c1 * p["G"] + c2 * q["G"]))
    wG = c1 * oracle.sigma(lib=lib, **p) + c2 * oracle.sigma(lib=lib, **dict(p, G=q["G"]))
    e = max(_rel(sD, wD), _rel(sG, wG))
    assert e < 1e-13, e
    return e


def pin_hand_example(lib=oracle.LIB):
    """A worked example small enough to do by hand: Norb = 2, one atom that is
    its own neighbour, Nkz = Nqz = 1, one frequency (s = 1), NE = 2,
    dH_x = [[1, 2], [0, 1]], dH_y = dH_z = 0, D~_xx = 2i, G(E=0) = [[i, 1], [-1, 2i]].
    dH_x G = [[i-2, 1+4i], [-1, 2i]];  (dH_x G) dH_x^T = [[9i, 1+4i], [-1+4i, 2i]];
    Sigma(E=1) = i * 2i * that = [[-18i, -2-8i], [2-8i, -4i]];  Sigma(E=0) = 0."""
    neigh = np.zeros((1, 1), dtype=np.int32)
    dH = np.zeros((1, 1, 3, 2, 2))
    dH[0, 0, 0] = [[1, 2], [0, 1]]
    G = np.zeros((1, 2, 1, 2, 2), dtype=np.complex128)
    G[0, 0, 0] = [[1j, 1], [-1, 2j]]
    G[0, 1, 0] = [[5, 5], [5, 5]]  # never read: E=1 - s = 0 and E=0 - s < 0
    D = np.zeros((1, 1, 1, 1, 3, 3), dtype=np.complex128)
    D[0, 0, 0, 0, 0, 0] = 2j
    got = oracle.sigma(neigh, dH, G, D, [1], 1, 2, alpha=1j, lib=lib)
    want = np.zeros((1, 2, 1, 2, 2), dtype=np.complex128)
    want[0, 1, 0] = [[-18j, -2 - 8j], [2 - 8j, -4j]]
    assert np.array_equal(got, want), got
    return 0.0


def pin_generated_inputs(lib=oracle.LIB):
    """The generated problem (the small CPU-scale configuration) obeys the
    anti-Hermitian symmetry and the edge pin too."""
    NA, NB, Norb, Nkz, Nqz, NE, Nw = 16, 4, 4, 3, 3, 64, 4
    shift = np.arange(1, Nw + 1, dtype=np.int32)
    neigh = ssegen.neigh(SEED, NA, NB)
    dH = ssegen.dH(SEED, NA, NB, Norb)
    G = ssegen.G(SEED, 0, Nkz, NE, NA, Norb)
    D = ssegen.D(SEED, 0, Nqz, Nw, NA, NB)
    s = oracle.sigma(neigh, dH, G, D, shift, Nkz, NE, alpha=1j, lib=lib)
    sh = np.conj(np.swapaxes(s, -1, -2))
    e = _ratio(s + sh, s)
    assert e < 1e-14, e
    assert np.array_equal(s[:, 0], np.zeros_like(s[:, 0]))
    return e


def _sampled_case():
    """A problem whose block list exercises the sampled evaluation: negative and
    unsorted shifts, kz wrap (k < Nqz - 1), the output energy edges 0,
    s_max - 1, s_max and NE - 1, reads of the top G energy (e = 9 with the
    shift -2), atoms 0 and NA - 1, and repeated, unsorted blocks."""
    rng = np.random.default_rng(21)
    p = small_problem(rng, NA=7, NB=3, Norb=3, Nkz=4, Nqz=3, NE=12, shift=(3, -2, 1, 5))
    smax = int(np.max(p["shift"]))
    blocks = [(0, 0, 0), (3, 11, 6), (0, smax - 1, 2), (1, smax, 6), (2, 11, 0),
              (0, 7, 3), (3, 0, 5), (1, 1, 1), (0, 7, 3), (2, 6, 4), (0, 0, 0), (3, smax, 1),
              (1, 9, 2)]
    return p, np.array(blocks, dtype=np.int32)


def pin_sampled_blocks(lib=oracle.LIB):
    """The sampled evaluation (a list of output blocks, and G supplied as a
    stack of only the blocks they read, located through gslot) reproduces the
    full evaluation bit for bit: each output block of Eq. (3) is a function of
    its own (k, e, a) and of G blocks that a flat row-major index names."""
    p, blocks = _sampled_case()
    Nkz, NE = p["Nkz"], p["NE"]
    NA, Norb = p["dH"].shape[0], p["dH"].shape[3]
    Nqz = p["D"].shape[0]
    full = oracle.sigma(lib=lib, **p)
    want = full[blocks[:, 0], blocks[:, 1], blocks[:, 2]]
    # blocks listed, full G
    got = oracle.sigma(lib=lib, blocks=blocks, **p)
    assert np.array_equal(got, want)
    # blocks listed, G as a stack of the needed blocks in a scrambled order
    need = oracle.needed_g_blocks(p["neigh"], p["shift"], Nkz, Nqz, NE, NA, blocks)
    order = np.random.default_rng(22).permutation(need.size)
    Gflat = p["G"].reshape(-1, Norb, Norb)   # row-major: flat index (k NE + e) NA + a
    stack = Gflat[need[order]]
    gslot = np.full(Nkz * NE * NA, -1, dtype=np.int64)
    gslot[need[order]] = np.arange(need.size)
    got2 = oracle.sigma(lib=lib, blocks=blocks, gslot=gslot, **dict(p, G=stack))
    assert np.array_equal(got2, want)
    return 0.0


def pin_needed_blocks_exact(lib=oracle.LIB):
    """needed_g_blocks names exactly the G blocks the listed outputs read:
    with every listed block supplied the evaluation succeeds and matches the
    full one (pin_sampled_blocks), and withholding any one of them is reported
    as a missing block, so no listed block is superfluous."""
    p, blocks = _sampled_case()
    Nkz, NE = p["Nkz"], p["NE"]
    NA, Norb = p["dH"].shape[0], p["dH"].shape[3]
    Nqz = p["D"].shape[0]
    need = oracle.needed_g_blocks(p["neigh"], p["shift"], Nkz, Nqz, NE, NA, blocks)
    assert np.unique(need).size == need.size
    Gflat = p["G"].reshape(-1, Norb, Norb)
    for drop in range(need.size):
        keep = np.delete(need, drop)
        gslot = np.full(Nkz * NE * NA, -1, dtype=np.int64)
        gslot[keep] = np.arange(keep.size)
        try:
            oracle.sigma(lib=lib, blocks=blocks, gslot=gslot, **dict(p, G=Gflat[keep]))
        except ValueError:
            continue
        raise AssertionError(f"block {need[drop]} withheld but not reported missing")
    return 0.0


ALL_PINS = [pin_single_term, pin_fft_correlation, pin_closed_form_constant, pin_antihermitian,
            pin_kz_roll, pin_energy_shift_and_edge, pin_atom_relabel, pin_linearity,
            pin_hand_example, pin_generated_inputs, pin_sampled_blocks,
            pin_needed_blocks_exact]
