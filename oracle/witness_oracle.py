"""FP64 CPU oracle of off-axis and transverse wakes from the 3-D TE/TM scheme (23).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product package;
it shares no code with the HIP path.

Sec. 5 defines the longitudinal wake potential by the integral of E_z along the
path of a witness particle that follows the bunch at distance s, normalised by
the bunch charge.  The explicit oracle (``oracle.run``) samples it on the
bunch's own node line.  Here the bunch stays on its line (i0, j0) and the
wake is sampled on other e_z node lines (i, j) with the same quadrature: step n
adds -1/2 (e_z^{n-1/2} + e_z^{n+1/2}) of edge k to sample s_j, j = n - k - M
(edge k is met at time tau = (k + M + j) dz, half way between the two levels).

The transverse wake follows from the Panofsky-Wenzel theorem.  With
W_par = -(1/Q) int E_z dz and W_perp = (1/Q) int (E + v x B)_perp dz along the
same path, Faraday's law gives d W_perp / ds = grad_perp W_par.  W_perp is
integrated over s from the first sample (ahead of the bunch, where no wake has
arrived) with the trapezoid rule; the gradient at the witness node is the
centred difference of its four neighbouring lines.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

# witness node and its four neighbours, in this order
OFFSETS = ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))


def witness_lines(iw: int, jw: int) -> list[tuple[int, int]]:
    return [(iw + di, jw + dj) for di, dj in OFFSETS]


def run(g: O.Geom, m: dict, f: dict, nsteps: int, bunch: O.Bunch, lines, n0: int = 0,
        acc: np.ndarray | None = None, src_acc: np.ndarray | None = None) -> dict:
    """Run nsteps steps of (23) with the bunch, in place, accumulating the wake
    quadrature on every (i, j) of ``lines``.  Returns dict(acc (len(lines), nw),
    src_acc (nw): the oracle's own bunch-line accumulator); W = acc / Q."""
    L = len(lines)
    if acc is None:
        acc = np.zeros((L, bunch.nw))
    if src_acc is None:
        src_acc = np.zeros(bunch.nw)
    k = np.arange(g.nz)
    for s in range(nsteps):
        n = n0 + s
        old = [f["ez"][i, j, : g.nz].copy() for i, j in lines]
        O.run(g, m, f, 1, n0=n, bunch=bunch, acc=src_acc)
        js = n - k - bunch.M
        ok = (js >= bunch.jmin) & (js < bunch.jmin + bunch.nw)
        if 0 < bunch.kend < g.nz:
            ok &= k < bunch.kend
        for l, (i, j) in enumerate(lines):
            new = f["ez"][i, j, : g.nz]
            # distinct edges of one step feed distinct samples
            acc[l, js[ok] - bunch.jmin] += -0.5 * (old[l][ok] + new[ok])
    return {"acc": acc, "src_acc": src_acc}


def pw_integral(D: np.ndarray, ds: float) -> np.ndarray:
    """Trapezoid rule int_{s_0}^{s_j} D ds', zero at the first sample."""
    out = np.zeros_like(D)
    out[1:] = np.cumsum(0.5 * (D[1:] + D[:-1])) * ds
    return out


def transverse_wake(acc5: np.ndarray, Q: float, dx: float, dy: float, ds: float):
    """(W_x, W_y) at the witness node from the five lines of ``run`` with
    ``witness_lines``: centred differences of W_par = acc / Q across the node,
    integrated over s."""
    W = acc5 / Q
    Dx = (W[2] - W[1]) / (2.0 * dx)
    Dy = (W[4] - W[3]) / (2.0 * dy)
    return pw_integral(Dx, ds), pw_integral(Dy, ds)
