"""Operation-count model of the paper's Section 4 (test infrastructure only).

With N = 2^m data and 2^l processors, each processor multiplies along its own
branch up to level m1 = m - l, which costs (m - l) 2^(m - l) products, and the
remaining l levels run on a halving number of processors, 2^(m - l + i) products
for i = 1..l (eq. multi).  The ratio of the sequential count m 2^m (= N log2 N)
to that parallel count is the paper's speed-up (RSP), tabulated in Table 1 for
four processors.
"""


def sequential_products(m: int) -> int:
    """N log2 N with N = 2^m (Section 2 / Table 1 column N Log2 N)."""
    return m * (1 << m)


def direct_products(m: int) -> int:
    """N^2 multiplications of the direct sum (Table 1 column N^2)."""
    return (1 << m) ** 2


def parallel_products(m: int, l: int) -> int:
    """Critical-path products of the parallel tree, eq. (multi)."""
    if not (0 <= l <= m):
        raise ValueError("need 0 <= l <= m")
    return (m - l) * (1 << (m - l)) + sum(1 << (m - l + i) for i in range(1, l + 1))


def speedup(m: int, l: int) -> float:
    """Sequential / parallel product ratio, m / ((m-l) 2^-l + sum_i 2^(i-l))."""
    return sequential_products(m) / parallel_products(m, l)
