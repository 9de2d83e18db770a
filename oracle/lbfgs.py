"""Textbook L-BFGS with a maximal step and Armijo backtracking, in FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle.py).  The paper's Methods hand the
configuration and the gradient to L-BFGS (Liu & Nocedal) with a cap on the
step length and a backtracking line search (Nocedal & Wright), and give no
constants for either.  The reading taken here: m stored pairs, no coordinate
moves farther than max_step in one step, Armijo sufficient decrease with
constant c1, backtracking by the factor shrink, and after max_backtracks
rejected trials the history is dropped and the search restarts along -g.  The
loss and gradient come from the direct-sum oracle (or any callable with the
same signature).

Two-loop recursion (Nocedal & Wright, Algorithm 7.4): with pairs (s_i, y_i),
rho_i = 1 / y_i.s_i,
  q = g;  for i newest..oldest: a_i = rho_i s_i.q;  q -= a_i y_i
  q *= gamma = s.y / y.y (newest pair)
  for i oldest..newest: b = rho_i y_i.q;  q += (a_i - b) s_i
  p = -q.
The recursion is written out in two_loop(), which run() calls for every
direction; the pins check it against the dense inverse-Hessian update.
"""
from __future__ import annotations

import numpy as np


def two_loop(g, S, Y, R, gamma):
    """H g for the limited-memory inverse Hessian H of the stored pairs (lists S,
    Y, R = 1/y.s, oldest first) with initial matrix gamma I (Nocedal & Wright,
    Algorithm 7.4).  With no pairs, H = I."""
    q = np.array(g, dtype=np.float64, copy=True)
    a = [0.0] * len(S)
    for i in range(len(S) - 1, -1, -1):
        a[i] = R[i] * float(S[i] @ q)
        q -= a[i] * Y[i]
    if S:
        q *= gamma
    for i in range(len(S)):
        b = R[i] * float(Y[i] @ q)
        q += (a[i] - b) * S[i]
    return q


def run(fg, x0, n_iter, m=8, max_step=0.1, c1=1e-4, shrink=0.5, max_backtracks=20, gtol=0.0,
        direction=two_loop):
    """fg(x) -> (f, g) on flat FP64 vectors; stops early when the RMS gradient is at
    most gtol.  direction(g, S, Y, R, gamma) returns H g (default: the two-loop
    recursion).  Returns dict(x, f, fs, nevals, xs)."""
    x = np.array(x0, dtype=np.float64).ravel().copy()
    f, g = fg(x)
    nevals = 1
    S, Y, R = [], [], []
    gamma = 1.0
    p = -g
    fs = [f]
    xs = [x.copy()]

    def step_len(p):
        pm = np.max(np.abs(p))
        return max_step / pm if pm > max_step else 1.0

    alpha = step_len(p)
    gtp = float(g @ p)
    restarted = False
    for _ in range(n_iter):
        if gtol > 0 and np.sqrt(float(g @ g) / g.size) <= gtol:
            break
        nbt = 0
        while True:
            xt = x + alpha * p
            ft, gt = fg(xt)
            nevals += 1
            if np.isfinite(ft) and ft <= f + c1 * alpha * gtp:
                break
            nbt += 1
            if nbt > max_backtracks:
                if S or not restarted:
                    S, Y, R = [], [], []
                    restarted = True
                    p = -g
                    gtp = float(g @ p)
                    alpha = step_len(p)
                    nbt = 0
                    continue
                raise RuntimeError("line search failed")
            alpha *= shrink
        s = alpha * p
        y = gt - g
        x, f, g = xt, ft, gt
        ys = float(y @ s)
        yy = float(y @ y)
        if ys > 0 and yy > 0:
            S.append(s)
            Y.append(y)
            R.append(1.0 / ys)
            gamma = ys / yy
            restarted = False
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
                R.pop(0)
        else:
            S, Y, R = [], [], []
        p = -direction(g, S, Y, R, gamma)
        gtp = float(g @ p)
        if not gtp < 0:
            S, Y, R = [], [], []
            p = -g
            gtp = float(g @ p)
        alpha = step_len(p)
        fs.append(f)
        xs.append(x.copy())
    return {"x": x, "f": f, "fs": fs, "xs": xs, "nevals": nevals}
