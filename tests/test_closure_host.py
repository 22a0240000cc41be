"""Host-side pieces of the closure pipeline (CPU only): the cube-symmetry
images used to multiply training pairs are exact symmetries of the NS
discretisation and of the fine-to-coarse filter, checked on the FP64 oracle."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2608_09615_amd import closure as C
from paper_2608_09615_amd import workloads as W

# a pure reflection, a pure axis swap, a rotation and a mixed element
PICKS = [((0, 1, 2), (True, False, False)), ((1, 0, 2), (False, False, False)),
         ((1, 2, 0), (False, True, False)), ((2, 0, 1), (True, True, True))]


def test_symmetry_list_is_the_cube_group():
    assert len(C.SYMMETRIES) == 48 and C.SYMMETRIES[0] == ((0, 1, 2), (False, False, False))
    a = np.random.Generator(np.random.PCG64(0)).normal(size=(1, 5 * 27))
    images = {C.apply_symmetry(a, 3, s).tobytes() for s in C.SYMMETRIES}
    assert len(images) == 48
    assert np.array_equal(C.apply_symmetry(a, 3, C.SYMMETRIES[0]), a)


@pytest.mark.parametrize("sym", PICKS)
def test_ns_residual_commutes_with_symmetry(oracle_lib, sym):
    """R(S u) = S R(u) for the compact NS residual on a periodic cube: any
    axis, flip or momentum-sign slip in the map breaks it."""
    nel, p = (3, 3, 3), 2
    n = p + 1
    lo, hi = W.tgv_domain()
    U = W.perturbed_tgv_state(nel, p, seed=3, noise=1e-3)
    prm = oracle_lib.make_params("ns")
    g = lambda A: C.apply_symmetry(A.reshape(1, 3, 3, 3, 5 * n ** 3), n, sym, lead=4).reshape(A.shape)
    R = oracle_lib.rhs_3d(U, nel, lo, hi, p, "compact", prm)
    RS = oracle_lib.rhs_3d(g(U), nel, lo, hi, p, "compact", prm)
    assert np.abs(RS - g(R)).max() < 1e-11 * np.abs(R).max()
    assert np.abs(g(U) - U).max() > 1e-3       # the map does move the state


@pytest.mark.parametrize("sym", PICKS)
def test_per_element_images_match_global_image(sym):
    nel, n = 4, 3
    U = np.random.Generator(np.random.PCG64(1)).normal(size=(nel ** 3, 5 * n ** 3))
    glob = C.apply_symmetry(U.reshape(1, nel, nel, nel, -1), n, sym, lead=4).reshape(nel ** 3, -1)
    loc = C.apply_symmetry(U, n, sym)
    w = np.random.Generator(np.random.PCG64(2)).normal(size=U.shape[1])
    assert np.allclose(np.sort(glob @ w), np.sort(loc @ w), rtol=0, atol=1e-12)


@pytest.mark.parametrize("sym", PICKS[:2])
def test_filter_commutes_with_symmetry(sym):
    p, r, nc = 2, 2, 2
    n = p + 1
    nf = r * nc
    Uf = np.random.Generator(np.random.PCG64(4)).normal(size=(nf ** 3, 5, n, n, n))
    g = lambda A, m: C.apply_symmetry(A.reshape(1, m, m, m, -1), n, sym, lead=4).reshape(A.shape)
    a = M.filter_state(g(Uf, nf), (nf,) * 3, p, r)
    b = g(M.filter_state(Uf, (nf,) * 3, p, r), nc)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_augment_layout():
    n = 2
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.normal(size=(7, 5 * n ** 3))
    T = rng.normal(size=(7, 5 * n ** 3))
    Xa, Ta = C.augment(X, T, n, 4, seed=9)
    assert Xa.shape == (28, X.shape[1]) and Ta.shape == (28, T.shape[1])
    assert np.array_equal(Xa[::4], X) and np.array_equal(Ta[::4], T)
    for i in range(7):
        imgs = {Xa[4 * i + j].tobytes() for j in range(4)}
        assert len(imgs) == 4                   # distinct symmetries per sample
        for j in range(1, 4):                   # pairs stay matched
            hit = [s for s in C.SYMMETRIES if np.array_equal(C.apply_symmetry(X[i:i + 1], n, s)[0], Xa[4 * i + j])]
            assert hit and np.array_equal(C.apply_symmetry(T[i:i + 1], n, hit[0])[0], Ta[4 * i + j])
    Xb, _ = C.augment(X, T, n, 4, seed=9)
    assert np.array_equal(Xa, Xb)
