"""Cost figures the paper reports next to its solves (host arithmetic only).

* C: non-zeros of the Cholesky-type factor, the unit diagonal counted
  (Section 6, Tables 1-2; C of ILU(0) equals (E + N)/2, the lower triangle of A).
* M1: multiplications per PCG iteration, eq. m1: M1 = 2C + E + 4N.
* M2: total multiplications, M1 times the iteration count.
* Algorithmic bytes of the kernels, i.e. what each step must move at minimum.
"""


def factor_size(nnz_strict: int, n: int) -> int:
    """C = strictly-triangular non-zeros + N (the unit diagonal)."""
    return int(nnz_strict) + int(n)


def m1(C: int, E: int, N: int) -> int:
    """Multiplications per PCG iteration, eq. m1."""
    return 2 * int(C) + int(E) + 4 * int(N)


def m2(C: int, E: int, N: int, iters: int) -> int:
    return m1(C, E, N) * int(iters)


def walk_step_bytes(deg: float) -> float:
    """Algorithmic bytes of one walk step from a node of `deg` neighbours: the row
    extent (two 4-byte offsets), the rank of the chosen node (4 bytes) and the row's
    transition entries (4-byte neighbour id + 4-byte threshold each)."""
    return 12.0 + 8.0 * deg


def pcg_iter_bytes(nnz_a: int, n: int, nnz_y: int, factor_bytes: int = 8) -> float:
    """Algorithmic HBM bytes of one PCG iteration: A once (8 B value + 4 B column per
    entry, 8 B row pointer per row), the factor twice (value + 4 B column per entry,
    8 B row pointer per row, D once per solve) and the vector passes of the iteration
    (11 reads/writes of n doubles)."""
    a = 12.0 * nnz_a + 8.0 * (n + 1)
    y = 2.0 * ((factor_bytes + 4.0) * nnz_y + 8.0 * (n + 1) + factor_bytes * n)
    return a + y + 11.0 * 8.0 * n
