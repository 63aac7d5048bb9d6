"""Pins of the oracle's multiplicative Schwarz smoothers (EM, FM; Sec. 3.1).

* EM_0 (element blocks, no overlap) in lexicographic order is block Gauss-Seidel:
  one forward sweep equals u + (D + L)^-1 (f - A u) with D + L the block lower
  triangle of A in that order, one backward sweep u + (D + U)^-1 (f - A u): a
  matrix splitting, computed here by dense solves, not patch by patch.
* Two steps of one call (forwards, then backwards) form a symmetric smoother:
  the iteration matrix E of f = 0 satisfies A E = E^T A, for EM and FM with and
  without overlap (with the orientation order reversed as well for FM).
* Every subdomain correction is an A-orthogonal projection of the error, so the
  energy norm of the error never grows within a sweep.
* Colour classes: two subdomains of one class share no node and no matrix
  entry (A[S_s, S_t] = 0), on Dirichlet and periodic grids whose counts are and
  are not multiples of the colour modulus; so the coloured order takes the same
  steps as the lexicographic one, only reordered.
The printed rates of Tables 2-4 are pinned in test_oracle_multigrid."""
import itertools

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from oracle import schwarz as sw


def _grid(dim, n, periodic, seed):
    rng = np.random.default_rng(seed)
    return synth.Grid(dim, tuple(rng.uniform(0.5, 1.5, size=k) for k in n), (periodic,) * dim)


def _level(g, P, smoother, overlap, order="lex"):
    h = mg.Hierarchy(g, synth.Method(P=P, smoother=smoother, overlap=overlap, order=order,
                                     beta=(0.0,) * g.dim))
    return h, h.levels[-1].smoother, h.levels[-1].A.toarray()


def _gidx(sm, sig):
    """Global lexicographic indices of a subdomain (patch array order)."""
    dim = sm.grid.dim
    shape = sm.shape
    strides = [1]
    for d in range(dim - 1):
        strides.append(strides[-1] * shape[dim - 1 - d])
    p1 = [sm.patch_1d(d, sig[d]) for d in range(dim)]
    out = np.zeros([len(p1[d].idx) for d in reversed(range(dim))], dtype=np.int64)
    for d in range(dim):
        sh = [1] * dim
        sh[dim - 1 - d] = -1
        out = out + (p1[d].idx * strides[d]).reshape(sh)
    return out.reshape(-1)


@pytest.mark.parametrize("dim,n,periodic", [(2, (3, 4), False), (2, (3, 4), True), (3, (2, 3, 2), False)])
def test_em0_is_block_gauss_seidel(dim, n, periodic):
    g = _grid(dim, n, periodic, 3)
    h, sm, A = _level(g, 3, "EM", "zero")
    blocks = [_gidx(sm, sig) for sig in sm.mult_order(-1)]
    perm = np.concatenate(blocks)
    Ap = A[np.ix_(perm, perm)]
    nb = len(blocks[0])
    lower = np.zeros_like(Ap)
    upper = np.zeros_like(Ap)
    for i in range(len(blocks)):
        for j in range(len(blocks)):
            blk = Ap[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            if j <= i:
                lower[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = blk
            if j >= i:
                upper[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = blk
    rng = np.random.default_rng(4)
    u, f = rng.standard_normal((2, A.shape[0]))
    r = (f - A @ u)[perm]
    fwd = u.copy()
    fwd[perm] += np.linalg.solve(lower, r)         # block triangular: dense solves
    bwd = u.copy()
    bwd[perm] += np.linalg.solve(upper, r)
    assert np.allclose(sm.msweep(u, f, -1, False), fwd, rtol=0, atol=1e-11 * np.abs(fwd).max())
    assert np.allclose(sm.msweep(u, f, -1, True), bwd, rtol=0, atol=1e-11 * np.abs(bwd).max())


@pytest.mark.parametrize("smoother,overlap,order", [("EM", "zero", "lex"), ("EM", "level", "lex"),
                                                    ("FM", "zero", "lex"), ("FM", "level", "colour")])
def test_two_steps_are_symmetric(smoother, overlap, order):
    g = _grid(2, (3, 3), False, 5)
    h, sm, A = _level(g, 4, smoother, overlap, order)
    n = A.shape[0]
    E = np.empty((n, n))
    z = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        E[:, k] = sm.smooth(e, z, 2)
    AE = A @ E
    assert np.abs(AE - AE.T).max() <= 1e-9 * np.abs(AE).max()
    E1 = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        E1[:, k] = sm.smooth(e, z, 1)
    AE1 = A @ E1
    assert np.abs(AE1 - AE1.T).max() > 1e-3 * np.abs(AE1).max()     # one sweep alone is not symmetric


@pytest.mark.parametrize("smoother,overlap", [("EM", "level"), ("FM", "level"), ("FM", "zero")])
def test_energy_of_the_error_never_grows(smoother, overlap):
    g = _grid(2, (3, 4), False, 6)
    h, sm, A = _level(g, 4, smoother, overlap)
    rng = np.random.default_rng(7)
    x_star = rng.standard_normal(A.shape[0])
    f = A @ x_star
    u = np.zeros_like(f)
    energies = []
    normals = [-1] if smoother == "EM" else [0, 1]
    for nd in normals:
        for sig in sm.mult_order(nd):
            idx = _gidx(sm, sig)
            rs = f[idx] - A[idx] @ u
            u[idx] += np.linalg.solve(A[np.ix_(idx, idx)], rs)
            e = u - x_star
            energies.append(e @ A @ e)
    assert np.all(np.diff(energies) <= 1e-9 * energies[0])
    e0 = x_star @ A @ x_star
    assert energies[-1] < 0.5 * e0


@pytest.mark.parametrize("n,periodic", [((3, 4), True), ((5, 3), True), ((4, 4), False), ((6, 5), True)])
@pytest.mark.parametrize("smoother,overlap", [("EM", "zero"), ("EM", "level"), ("FM", "zero"), ("FM", "level")])
def test_colour_classes_are_independent(n, periodic, smoother, overlap):
    g = _grid(2, n, periodic, 8)
    h, sm, A = _level(g, 4, smoother, overlap, order="colour")
    normals = [-1] if smoother == "EM" else [0, 1]
    for nd in normals:
        counts = [len(sm.fc[d]) if d == nd else len(sm.ec[d]) for d in range(2)]
        classes = {}
        for sig in sm.mult_order(nd):
            key = tuple(sw.colour_digit(sig[d][1], counts[d], sw.colour_modulus(sm.n_o, d == nd), periodic)
                        for d in range(2))
            classes.setdefault(key, []).append(_gidx(sm, sig))
        assert len(classes) > 1
        for members in classes.values():
            for a, b in itertools.combinations(members, 2):
                assert not set(a) & set(b)
                assert np.all(A[np.ix_(a, b)] == 0.0)
        assert sum(len(v) for v in classes.values()) == np.prod(counts)


def test_colour_order_is_a_reordering():
    """The coloured sweep visits the same subdomains, in colour-major order."""
    g = _grid(2, (6, 4), True, 9)
    _, sl, _ = _level(g, 4, "FM", "level", "lex")
    _, sc, _ = _level(g, 4, "FM", "level", "colour")
    for nd in (0, 1):
        a, b = sl.mult_order(nd), sc.mult_order(nd)
        assert sorted(a) == sorted(b) and a != b
