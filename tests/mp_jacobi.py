"""Cyclic Jacobi eigenvalue method in mpmath (Golub and Van Loan, Sec. 8.5).

A brute-force high-precision reference: it returns the eigenpairs of the
stored double-precision matrix to about `dps` decimal digits, independent of
the refinement method and of the oracle.  Practical for n up to a few dozen.
"""
import mpmath


def jacobi_eigh(A, dps=40, sweeps=30):
    n = len(A)
    with mpmath.workdps(dps):
        a = [[mpmath.mpf(float(A[i][j])) for j in range(n)] for i in range(n)]
        v = [[mpmath.mpf(1) if i == j else mpmath.mpf(0) for j in range(n)] for i in range(n)]
        tol = mpmath.mpf(10) ** (-dps + 2)
        for _ in range(sweeps):
            off = mpmath.fsum(a[i][j] ** 2 for i in range(n) for j in range(n) if i != j)
            if off < tol ** 2:
                break
            for p in range(n - 1):
                for q in range(p + 1, n):
                    if a[p][q] == 0:
                        continue
                    theta = (a[q][q] - a[p][p]) / (2 * a[p][q])
                    t = mpmath.sign(theta) / (abs(theta) + mpmath.sqrt(theta ** 2 + 1))
                    if theta == 0:
                        t = mpmath.mpf(1)
                    c = 1 / mpmath.sqrt(t ** 2 + 1)
                    s = t * c
                    for r in range(n):            # A <- A J (columns p, q)
                        arp, arq = a[r][p], a[r][q]
                        a[r][p] = c * arp - s * arq
                        a[r][q] = s * arp + c * arq
                    for r in range(n):            # A <- J^T A (rows p, q)
                        apr, aqr = a[p][r], a[q][r]
                        a[p][r] = c * apr - s * aqr
                        a[q][r] = s * apr + c * aqr
                    for r in range(n):            # V <- V J
                        vrp, vrq = v[r][p], v[r][q]
                        v[r][p] = c * vrp - s * vrq
                        v[r][q] = s * vrp + c * vrq
        lam = [a[i][i] for i in range(n)]
        return lam, v
