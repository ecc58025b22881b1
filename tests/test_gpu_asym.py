"""Parity of the asymmetric path (Section 7.1) on the HIP side with the CPU oracle:
both games' factors bit-exact (the game of A^T is built from A^T with the ordering of
the game of A), one preconditioner application within 1e-12, BiCGSTAB with the same
iteration count and iterates within 1e-10."""
import numpy as np
import pytest

import oracle as O
from paper_math_0609672_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def srw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_math_0609672_amd import srw as s
    return s


DEV = "cuda:0"


def np_(t):
    return t.detach().cpu().numpy()


def random_asym(n, edges, seed):
    base = W.random_graph(n, edges, seed=seed, ground_frac=0.02)
    S = base.to_scipy().tocoo()
    m = S.row < S.col
    rng = np.random.default_rng(seed + 1)
    g = -S.data[m]
    t = rng.uniform(-0.7, 0.7, g.size)
    exc = np.zeros(n)
    exc[rng.choice(n, max(1, n // 50), replace=False)] = rng.uniform(0.1, 1.0, max(1, n // 50))
    return W.assemble_directed(n, S.row[m], S.col[m], g * (1 + t), g * (1 - t), exc)


CASES = {
    "grid2d_asym_30x23": (W.grid_asym((30, 23), g=("uniform", 0.1, 10.0), skew=0.6, ground_frac=0.02,
                                      excess=("uniform", 0.1, 10.0), seed=3), 64),
    "grid3d_asym_12": (W.grid_asym((12, 12, 12), g=("loguniform", 1e-2, 1e2), skew=0.5,
                                   ground_frac=0.01, excess=("uniform", 0.01, 1.0), seed=4), 96),
    "random_asym_2500": (random_asym(2500, 8000, 9), 40),
}


def export(F):
    return {k: np_(v) for k, v in F.export().items()}


def same_factor(got, ref):
    assert np.array_equal(got["yptr"], ref.yptr)
    assert np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval)
    assert np.array_equal(got["d"], ref.d)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("drop", [0.0, 1e-3])
def test_two_game_factors_bit_exact(srw, name, drop):
    A, walks = CASES[name]
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, walks, drop, 5)
    ref = O.build_factor_ldu(A, walks, drop, 5)
    got_a, got_t = export(F), export(F.transpose_game())
    assert np.array_equal(got_a["rank"], ref.a.rank) and np.array_equal(got_t["rank"], ref.a.rank)
    same_factor(got_a, ref.a)
    same_factor(got_t, ref.t)
    assert F.stats()["two_game"] == 1


def test_symmetric_input_gives_one_factor_twice(srw):
    A = W.config_grid2d_32(0)
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, 32, 1e-3, 2)
    # the two-game solves substitute every row: bit for bit against the symmetric
    # factor without the dense head, to rounding against it with the head
    P = srw.build_factor(Mx, 32, 1e-3, 2, head_rows=-1)
    Ph = srw.build_factor(Mx, 32, 1e-3, 2)
    a, t, p = export(F), export(F.transpose_game()), export(P)
    for k in ("yptr", "ycol", "yval", "d"):
        assert np.array_equal(a[k], t[k]) and np.array_equal(a[k], p[k])
    r = torch.randn(A.n, dtype=torch.float64, device=DEV)
    z = srw.apply(F, r)
    assert torch.equal(z, srw.apply(P, r))
    assert float(torch.linalg.norm(srw.apply(Ph, r) - z)) <= 1e-13 * float(torch.linalg.norm(z))


@pytest.mark.parametrize("name", list(CASES))
def test_ldu_apply_matches_oracle(srw, name):
    A, walks = CASES[name]
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, walks, 1e-4, 6)
    ref = O.build_factor_ldu(A, walks, 1e-4, 6)
    r = np.random.default_rng(3).standard_normal(A.n)
    z = np_(srw.apply(F, torch.as_tensor(r, device=DEV)))
    zr = O.apply_ldu(ref, r)
    assert np.allclose(z, zr, rtol=1e-12, atol=1e-12 * np.abs(zr).max())


@pytest.mark.parametrize("name", list(CASES))
def test_bicgstab_matches_oracle(srw, name):
    A, walks = CASES[name]
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, walks, 1e-4, 7)
    ref = O.build_factor_ldu(A, walks, 1e-4, 7)
    b = np.random.default_rng(4).standard_normal(A.n)
    st, x, it, rel = srw.bicgstab_solve(Mx, F, torch.as_tensor(b, device=DEV), 1e-10)
    rst, rx, rit, rrel = O.bicgstab(A, ref, b, 1e-10)
    assert st == rst == 0 and it == rit and rel <= 1e-10
    assert np.allclose(np_(x), rx, rtol=1e-10, atol=1e-10 * np.abs(rx).max())


@pytest.mark.parametrize("name", list(CASES))
def test_unpreconditioned_bicgstab(srw, name):
    """Without a preconditioner the method runs hundreds of iterations on these
    matrices and the last-bit differences of the dot products (summed in another order
    on the GPU) grow: the first iterates agree to 1e-9, both runs converge, and their
    iteration counts agree within 10 %."""
    A, _ = CASES[name]
    Mx = srw.Matrix.from_host(A, DEV)
    b = np.random.default_rng(4).standard_normal(A.n)
    bt = torch.as_tensor(b, device=DEV)
    for k in (1, 4, 8):
        _, x, it, _ = srw.bicgstab_solve(Mx, None, bt, 0.0, k)
        _, rx, rit, _ = O.bicgstab(A, None, b, 0.0, k)
        assert it == rit == k
        assert np.allclose(np_(x), rx, rtol=1e-9, atol=1e-9 * np.abs(rx).max())
    st, x, it, rel = srw.bicgstab_solve(Mx, None, bt, 1e-10, 5000)
    rst, rx, rit, rrel = O.bicgstab(A, None, b, 1e-10, 5000)
    assert st == rst == 0 and rel <= 1e-10 and rrel <= 1e-10
    assert abs(it - rit) <= 0.1 * rit + 2


def test_bicgstab_iterates_match_oracle(srw):
    A, walks = CASES["grid3d_asym_12"]
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, walks, 1e-4, 8)
    ref = O.build_factor_ldu(A, walks, 1e-4, 8)
    b = np.random.default_rng(5).standard_normal(A.n)
    for k in (1, 2, 3, 5):
        st, x, it, _ = srw.bicgstab_solve(Mx, F, torch.as_tensor(b, device=DEV), 0.0, k)
        rst, rx, rit, _ = O.bicgstab(A, ref, b, 0.0, k)
        assert st == rst == 1 and it == rit == k
        assert np.allclose(np_(x), rx, rtol=1e-10, atol=1e-10 * np.abs(rx).max())


def test_two_game_options(srw):
    A, walks = CASES["grid2d_asym_30x23"]
    Mx = srw.Matrix.from_host(A, DEV)
    # walk reuse in both games
    F = srw.build_factor_ldu(Mx, 16, 1e-3, 3, reuse=True)
    ref = O.build_factor_ldu(A, 16, 1e-3, 3, reuse=True)
    same_factor(export(F), ref.a)
    same_factor(export(F.transpose_game()), ref.t)
    # FP32 factors: the FP64 ones rounded once, BiCGSTAB still reaches the tolerance
    G = srw.build_factor_ldu(Mx, walks, 1e-3, 3, precision="fp32")
    ref = O.build_factor_ldu(A, walks, 1e-3, 3)
    assert np.array_equal(export(G)["yval"], ref.a.yval.astype(np.float32))
    assert np.array_equal(export(G.transpose_game())["yval"], ref.t.yval.astype(np.float32))
    b = torch.ones(A.n, dtype=torch.float64, device=DEV)
    st, _, it, rel = srw.bicgstab_solve(Mx, G, b, 1e-10)
    assert st == 0 and rel <= 1e-10


def test_errors(srw):
    A, _ = CASES["grid2d_asym_30x23"]
    Mx = srw.Matrix.from_host(A, DEV)
    with pytest.raises(srw.SrwError) as e:
        srw.build_factor(Mx, 8, 0.0, 1)  # values not symmetric
    assert e.value.status == srw.E_NOT_RMATRIX
    F = srw.build_factor_ldu(Mx, 8, 0.0, 1)
    b = torch.ones(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(srw.SrwError) as e:
        srw.pcg_solve(Mx, F, b, 1e-8)
    assert e.value.status == srw.E_ARG
    P = srw.build_factor(srw.Matrix.from_host(W.config_grid2d_32(0), DEV), 8, 0.0, 1)
    with pytest.raises(srw.SrwError):
        P.transpose_game()
    # a column sum above the diagonal (rows still dominant)
    D = A.dense()
    j = 7
    i = next(i for i in range(A.n) if i != j and D[i, j] != 0)
    D[i, j] -= 50.0
    D[i, i] += 50.0
    with pytest.raises(srw.SrwError) as e:
        srw.build_factor_ldu(srw.Matrix.from_host(W.from_dense(D), DEV), 8, 0.0, 1)
    assert e.value.status == srw.E_NOT_RMATRIX
    # a structurally asymmetric entry
    C = A.dense()
    i, j = np.argwhere(C == 0)[0]
    C[i, j] = -1e-3
    C[i, i] += 1.0
    C[j, j] += 1.0
    with pytest.raises(srw.SrwError) as e:
        srw.build_factor_ldu(srw.Matrix.from_host(W.from_dense(C), DEV), 8, 0.0, 1)
    assert e.value.status == srw.E_NOT_RMATRIX


def test_at_scale_64(srw):
    """3D asymmetric grid 64^3: BiCGSTAB with the two-game factor reaches 1e-8 on the
    true residual in far fewer iterations than without it."""
    A = W.config_grid3d_asym(64, 0)
    Mx = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor_ldu(Mx, 64, 1e-4, 0)
    b = torch.as_tensor(W.rhs(A.n, seed=0), device=DEV)
    st, x, it, rel = srw.bicgstab_solve(Mx, F, b, 1e-8)
    st0, _, it0, rel0 = srw.bicgstab_solve(Mx, None, b, 1e-8, 5000)
    assert st == 0 and rel <= 1e-8
    assert it * 4 < it0
