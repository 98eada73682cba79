"""Recommended search settings per target recall (Section 4.4, Table 3).

Each row gives the coarse candidate count N_c, the re-rank depth N_rerank,
the early-termination thresholds (gap, ratio) and the ef multiplier m_ef.
Section 3.2 searches with ef = N_c * m_ef, so a row also fixes ef.
"""

# (lower end of the row's recall range, N_c, N_rerank, tau_gap, tau_ratio, m_ef)
TABLE3 = (
    (0.85, 35, 12, 0.020, 1.015, 2),
    (0.90, 45, 16, 0.015, 1.012, 2),
    (0.95, 55, 20, 0.012, 1.010, 3),
    (0.97, 70, 28, 0.010, 1.008, 3),
)


def table3(target):
    """Settings of the Table 3 row for a target recall: the last row whose
    range starts at or below the target (the first row below 0.85).
    Returns dict(ef, nc, n_rerank, tau_gap, tau_ratio, m_ef), the keyword
    arguments of a query plan plus ef and N_c."""
    row = TABLE3[0]
    for r in TABLE3:
        if target >= r[0]:
            row = r
    lo, nc, nrr, gap, ratio, m_ef = row
    return dict(ef=nc * m_ef, nc=nc, n_rerank=nrr, tau_gap=gap, tau_ratio=ratio, m_ef=m_ef)
