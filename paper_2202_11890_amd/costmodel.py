"""Work counting for MPRK vs single-rate Runge-Kutta (Section 4, performance
analysis, eq. speedup and eq. par_speedup).

A *cell-stage update* is one right-hand-side evaluation plus its stage
combination at one cell.  Per slow step of size dt, MPRK with an s-stage base
method and rate m evaluates the slow region s times and the buffer and fast
regions m*s times; the single-rate method at step dt/m evaluates every cell
m*s times.
"""
from __future__ import annotations


def mprk_cell_stages(n_fast: int, n_buffer: int, n_slow: int, m: int, s: int) -> int:
    """s N_S + m s N_B + m s N_F (Section 4, serial case)."""
    return s * n_slow + m * s * (n_buffer + n_fast)


def sr_cell_stages(n_total: int, m: int, s: int) -> int:
    """m s N_total: single-rate steps of dt/m over one slow step."""
    return m * s * n_total


def speedup(slow_fraction: float, m: int) -> float:
    """eq. speedup: (1 + (1/m - 1) N_S / N_total)^-1.  With per-process counts
    N_S,EPS / N_total,EPS it is eq. par_speedup."""
    return 1.0 / (1.0 + (1.0 / m - 1.0) * slow_fraction)


def speedup_from_counts(n_fast: int, n_buffer: int, n_slow: int, m: int, s: int = 2) -> float:
    total = n_fast + n_buffer + n_slow
    return sr_cell_stages(total, m, s) / mprk_cell_stages(n_fast, n_buffer, n_slow, m, s)


def partition_counts(nx: int, nz_fast: int, nz_slow: int, n_buffer: int, ny: int = 1):
    """(N_F, N_B, N_S) for stacked domains whose buffer is the n_buffer slow
    rows next to the interface."""
    col = nx * ny
    return col * nz_fast, col * n_buffer, col * (nz_slow - n_buffer)


def state_bytes_per_cell_stage(nv: int, s: int, word: int = 8) -> float:
    """Algorithmic HBM bytes per cell-stage for a low-storage stage update:
    each stage reads its stage value, reads the substep base (all stages but
    the first of a substep) and writes the next value: nv*word*(3 - 1/s)."""
    return nv * word * (3.0 - 1.0 / s)


def algorithmic_bytes_per_step(n_fast: int, n_buffer: int, n_slow: int, m: int, s: int,
                               nv: int = 4, word: int = 8) -> int:
    """Minimum HBM bytes one slow step must move: the per-stage state traffic
    of every evaluated cell, plus the buffer accumulator (written at the end
    of substep 1, read and written at substeps 2..m-1, read at substep m).
    Halo re-reads are implementation overhead and are not counted."""
    per_sub = nv * word * (2 + 3 * (s - 1))  # one s-stage substep for one cell
    fast = n_fast * m * per_sub
    slow = n_slow * per_sub
    buf = n_buffer * m * per_sub
    if m > 1:
        buf += n_buffer * nv * word * (1 + 2 * (m - 2) + 1)
    return fast + slow + buf
