"""FP64 CPU oracle for the FReSCo loss, structure factor and position gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()`` and
by the ``cpu_baseline`` leg of ``bench.py``.  The product library never uses it,
and this module shares no code with the HIP path (it does not import the
product package; the product package does not import it).

The arithmetic lives in ``oracle.c`` (direct sums from the definitions, see the
header there); this module marshals numpy arrays and turns the dense mode-cube
description of a problem (targets S0 and weights w on every integer mode
vector n with |n_a| <= M, C order, n_a running from -M to M) into the explicit
list of constrained modes that the sums run over.

Weight convention (Methods, "Analytical gradients"): the loss is
``sum_k W(k) (S(k) - S0(k))^2`` with ``W = w / S0^2`` where ``S0 != 0`` and
``W = w`` otherwise when the relative loss of Eq. (loss) is asked for
(``relative=True``); with ``relative=False`` the weights are used as given.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: an alternative build of oracle.c to load (the host-sanitizer run
# of the tests uses one); by default liboracle.so beside this file
_BUILT_SO = os.path.join(_HERE, "liboracle.so")
_SO = os.environ.get("ORACLE_LIB") or _BUILT_SO
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, portable x86-64 code)."""
    if force or not os.path.exists(_BUILT_SO):
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
               os.path.join(_HERE, "oracle.c"), "-o", _BUILT_SO + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_BUILT_SO + ".tmp", _BUILT_SO)
    return _BUILT_SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        ll = ctypes.c_longlong
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_rho.argtypes = [ctypes.c_int, ll, dp, dp, ll, ip, dp]
        lib.oracle_rho.restype = ctypes.c_int
        lib.oracle_loss_grad.argtypes = [ctypes.c_int, ll, dp, dp, ll, ip, dp, dp, dp, dp, dp,
                                         ll, lp, dp]
        lib.oracle_loss_grad.restype = ctypes.c_int
        lib.oracle_fd.argtypes = [ctypes.c_int, ll, dp, dp, ll, ip, dp, dp, ll, lp, ip,
                                  ctypes.c_double, dp]
        lib.oracle_fd.restype = ctypes.c_int
        lib.oracle_loss_grad_rho.argtypes = [ctypes.c_int, ll, dp, ll, ip, dp, dp, dp, dp, dp,
                                             ll, dp, dp]
        lib.oracle_loss_grad_rho.restype = ctypes.c_int
        lib.oracle_rho_direct.argtypes = [ctypes.c_int, ll, dp, dp, ll, ip, dp]
        lib.oracle_rho_direct.restype = ctypes.c_int
        lib.oracle_sf_vjp.argtypes = [ctypes.c_int, ll, dp, dp, ll, ip, dp, ll, lp, dp]
        lib.oracle_sf_vjp.restype = ctypes.c_int
        for f in (lib.oracle_pair, lib.oracle_pair_cells):
            f.argtypes = [ctypes.c_int, ll, dp, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, dp, dp]
            f.restype = ctypes.c_int
        lib.oracle_pair_fd.argtypes = [ctypes.c_int, ll, dp, dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ll, lp, ip, ctypes.c_double, dp]
        lib.oracle_pair_fd.restype = ctypes.c_int
        lib.oracle_rho_q.argtypes = [ctypes.c_int, ll, dp, dp, ll, dp, dp]
        lib.oracle_rho_q.restype = ctypes.c_int
        lib.oracle_loss_grad_q.argtypes = [ctypes.c_int, ll, dp, dp, ll, dp, dp, dp, dp, dp, dp]
        lib.oracle_loss_grad_q.restype = ctypes.c_int
        lib.oracle_grad_c_q.argtypes = [ctypes.c_int, ll, dp, dp, ll, dp, dp, dp, dp]
        lib.oracle_grad_c_q.restype = ctypes.c_int
        lib.oracle_rho_c.argtypes = [ctypes.c_int, ll, dp, dp, dp, ll, ip, dp]
        lib.oracle_rho_c.restype = ctypes.c_int
        lib.oracle_loss_grad_c.argtypes = [ctypes.c_int, ll, dp, dp, dp, ll, ip, dp, dp, dp, dp,
                                           ll, lp, dp, dp]
        lib.oracle_loss_grad_c.restype = ctypes.c_int
        lib.oracle_fd_c.argtypes = [ctypes.c_int, ll, dp, dp, dp, ll, ip, dp, dp, ll, lp, ip,
                                    ctypes.c_double, dp]
        lib.oracle_fd_c.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def threads() -> int:
    return int(_load().oracle_threads())


def _box(L, d):
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (d,))
    return np.ascontiguousarray(L, dtype=np.float64)


def _pos(pos):
    pos = np.asarray(pos)
    if pos.ndim != 2:
        raise ValueError("positions must be [N][d]")
    return np.ascontiguousarray(pos, dtype=np.float64)  # fp32 -> fp64 is exact


def _extent(d, M):
    return [int(m) for m in np.broadcast_to(np.asarray(M, dtype=np.int64), (d,))]


def mode_vectors(d: int, M) -> np.ndarray:
    """All integer mode vectors of the cube, C order, n_a = -M_a..M_a (M an int or
    one value per dimension): [prod (2M_a+1)][d]."""
    axes = [np.arange(-m, m + 1, dtype=np.int32) for m in _extent(d, M)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int32)


def effective_weights(w, S0, relative: bool):
    """W = w / S0^2 where S0 != 0 (relative loss, Eq. loss), else w."""
    w = np.asarray(w, dtype=np.float64)
    S0 = np.asarray(S0, dtype=np.float64)
    if not relative:
        return w.copy()
    W = w.copy()
    nz = S0 != 0
    W[nz] = w[nz] / (S0[nz] * S0[nz])
    return W


def constrained_set(d: int, M, w_cube, S0_cube, relative: bool = False):
    """Explicit constrained set from dense cubes: modes with w != 0 (the k = 0 mode is
    never part of the set).  Returns (modes [K][d] int32, W [K], S0 [K])."""
    n = mode_vectors(d, M)
    w = np.asarray(w_cube, dtype=np.float64).reshape(-1)
    S0 = np.zeros_like(w) if S0_cube is None else np.asarray(S0_cube, dtype=np.float64).reshape(-1)
    keep = (w != 0) & np.any(n != 0, axis=1)
    W = effective_weights(w[keep], S0[keep], relative)
    return np.ascontiguousarray(n[keep]), np.ascontiguousarray(W), np.ascontiguousarray(S0[keep])


def rho(pos, L, modes) -> np.ndarray:
    """rho(k) = sum_j exp(+i k.r_j) for the listed integer modes (k = 2 pi n / L)."""
    pos = _pos(pos)
    N, d = pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    out = np.zeros((modes.shape[0], 2), dtype=np.float64)
    st = _load().oracle_rho(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double),
                            modes.shape[0], _p(modes, ctypes.c_int), _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle_rho failed ({st})")
    return out[:, 0] + 1j * out[:, 1]


def structure_factor(pos, L, modes) -> np.ndarray:
    """S(k) = |rho(k)|^2 / N (Eq. structure_factor)."""
    r = rho(pos, L, modes)
    return (r.real ** 2 + r.imag ** 2) / np.asarray(pos).shape[0]


def structure_factor_cube(pos, L, M) -> np.ndarray:
    """S on the full mode cube prod (2M_a+1), C order, including S(0) = N."""
    d = np.asarray(pos).shape[1]
    S = structure_factor(pos, L, mode_vectors(d, M))
    return S.reshape(tuple(2 * m + 1 for m in _extent(d, M)))


def loss_grad(pos, L, modes, W, S0, grad_points=None, want_grad: bool = True):
    """Loss, structure factor on the listed modes and the gradient.

    grad_points: None for every point, or an index array for a subset.
    Returns dict(loss, S, rho, grad)."""
    pos = _pos(pos)
    N, d = pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = modes.shape[0]
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(K)
    S0 = np.ascontiguousarray(S0, dtype=np.float64).reshape(K)
    S = np.zeros(K)
    rh = np.zeros((K, 2))
    loss = np.zeros(1)
    if not want_grad:
        G, gidx, grad = 0, None, None
    elif grad_points is None:
        G, gidx = N, None
        grad = np.zeros((N, d))
    else:
        gidx = np.ascontiguousarray(grad_points, dtype=np.int64)
        G = gidx.shape[0]
        grad = np.zeros((G, d))
    st = _load().oracle_loss_grad(
        d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double), K,
        _p(modes, ctypes.c_int), _p(W, ctypes.c_double), _p(S0, ctypes.c_double),
        _p(S, ctypes.c_double), _p(rh, ctypes.c_double), _p(loss, ctypes.c_double), G,
        _p(gidx, ctypes.c_longlong), _p(grad, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle_loss_grad failed ({st})")
    return {"loss": float(loss[0]), "S": S, "rho": rh[:, 0] + 1j * rh[:, 1], "grad": grad}


def finite_difference(pos, L, modes, W, S0, coords, h: float) -> np.ndarray:
    """Central differences (L(r + h e) - L(r - h e)) / (2h) for coordinates
    coords = [(j, a), ...], evaluated without cancellation (see oracle.c)."""
    pos = _pos(pos)
    N, d = pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = modes.shape[0]
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, 2)
    cj = np.ascontiguousarray(coords[:, 0], dtype=np.int64)
    ca = np.ascontiguousarray(coords[:, 1], dtype=np.int32)
    out = np.zeros(coords.shape[0])
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(K)
    S0 = np.ascontiguousarray(S0, dtype=np.float64).reshape(K)
    st = _load().oracle_fd(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double), K,
                           _p(modes, ctypes.c_int), _p(W, ctypes.c_double),
                           _p(S0, ctypes.c_double), coords.shape[0],
                           _p(cj, ctypes.c_longlong), _p(ca, ctypes.c_int), float(h),
                           _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle_fd failed ({st})")
    return out


def sf_vjp(pos, L, modes, gS, grad_points=None) -> np.ndarray:
    """sum over the listed modes of gS(k) dS(k)/dr_j (derivative of S, Methods,
    "Analytical gradients"): the backward of r -> S for a given dF/dS.
    Returns [N][d] (or [len(grad_points)][d])."""
    pos = _pos(pos)
    N, d = pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = modes.shape[0]
    gS = np.ascontiguousarray(gS, dtype=np.float64).reshape(K)
    if grad_points is None:
        G, gidx = N, None
    else:
        gidx = np.ascontiguousarray(grad_points, dtype=np.int64)
        G = gidx.shape[0]
    grad = np.zeros((G, d))
    st = _load().oracle_sf_vjp(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double), K,
                               _p(modes, ctypes.c_int), _p(gS, ctypes.c_double), G,
                               _p(gidx, ctypes.c_longlong), _p(grad, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle_sf_vjp failed ({st})")
    return grad


def pair(pos, L, sigma: float, eps: float = 1.0, alpha: float = 2.0, cells: bool = False):
    """Soft-core repulsion U = (eps/alpha)(1 - r/sigma)^alpha for r < sigma under the
    minimum image: returns (energy, dE/dr [N][d]).  cells=False sums over all pairs,
    cells=True over a cell list (same sums, O(N))."""
    pos = _pos(pos)
    N, d = pos.shape
    e = np.zeros(1)
    grad = np.zeros((N, d))
    f = _load().oracle_pair_cells if cells else _load().oracle_pair
    st = f(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double), float(sigma),
           float(eps), float(alpha), _p(e, ctypes.c_double), _p(grad, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle pair term failed ({st})")
    return float(e[0]), grad


def _strengths(c, N):
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).ravel())
    if c.size != N:
        raise ValueError("one strength per point")
    return c


def rho_strengths(pos, c, L, modes) -> np.ndarray:
    """rho(k) = sum_j c_j exp(+i k.r_j) (Methods, Eq. ft) for the listed modes."""
    pos = _pos(pos)
    N, d = pos.shape
    c = _strengths(c, N)
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    out = np.zeros((len(modes), 2))
    st = _load().oracle_rho_c(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double),
                              _p(c, ctypes.c_double), len(modes), _p(modes, ctypes.c_int),
                              _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle rho with strengths failed ({st})")
    return out[:, 0] + 1j * out[:, 1]


def loss_grad_strengths(pos, c, L, modes, W, S0, grad_points=None, want_grad: bool = True):
    """Loss with real strengths c (S = |rho|^2 / rho0, rho0 = sum c^2) and its gradients
    with respect to positions and strengths (Methods, Eqs. losspositiongradient and
    lossweightgradient).  Returns dict(S, loss, grad [G][d], grad_c [G])."""
    pos = _pos(pos)
    N, d = pos.shape
    c = _strengths(c, N)
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = len(modes)
    W = np.ascontiguousarray(W, dtype=np.float64)
    S0 = np.ascontiguousarray(S0, dtype=np.float64)
    S = np.zeros(K)
    loss = np.zeros(1)
    if not want_grad:
        G, gidx = 0, None
    elif grad_points is None:
        G, gidx = N, None
    else:
        gidx = np.ascontiguousarray(grad_points, dtype=np.int64)
        G = len(gidx)
    grad = np.zeros((max(G, 1), d))
    grad_c = np.zeros(max(G, 1))
    st = _load().oracle_loss_grad_c(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double),
                                    _p(c, ctypes.c_double), K, _p(modes, ctypes.c_int),
                                    _p(W, ctypes.c_double), _p(S0, ctypes.c_double),
                                    _p(S, ctypes.c_double), _p(loss, ctypes.c_double), G,
                                    _p(gidx, ctypes.c_longlong), _p(grad, ctypes.c_double),
                                    _p(grad_c, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle loss with strengths failed ({st})")
    return {"S": S, "loss": float(loss[0]), "grad": grad[:G], "grad_c": grad_c[:G]}


def finite_difference_strengths(pos, c, L, modes, W, S0, coords, h: float) -> np.ndarray:
    """Cancellation-free central differences of the loss with strengths: coords
    [(j, a), ...] with a < d a position coordinate and a = d the strength c_j."""
    pos = _pos(pos)
    N, d = pos.shape
    c = _strengths(c, N)
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    W = np.ascontiguousarray(W, dtype=np.float64)
    S0 = np.ascontiguousarray(S0, dtype=np.float64)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, 2)
    cj = np.ascontiguousarray(coords[:, 0], dtype=np.int64)
    ca = np.ascontiguousarray(coords[:, 1], dtype=np.int32)
    out = np.zeros(len(coords))
    st = _load().oracle_fd_c(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double),
                             _p(c, ctypes.c_double), len(modes), _p(modes, ctypes.c_int),
                             _p(W, ctypes.c_double), _p(S0, ctypes.c_double), len(coords),
                             _p(cj, ctypes.c_longlong), _p(ca, ctypes.c_int), float(h),
                             _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle finite difference with strengths failed ({st})")
    return out


def rho_q(pos, q, c=None) -> np.ndarray:
    """rho(q) = sum_j c_j exp(+i q.r_j) at arbitrary wave vectors q [K][d] (free
    boundary conditions: positions as given), by direct sums."""
    pos = _pos(pos)
    N, d = pos.shape
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, d))
    cc = None if c is None else _strengths(c, N)
    out = np.zeros((len(q), 2))
    st = _load().oracle_rho_q(d, N, _p(pos, ctypes.c_double), _p(cc, ctypes.c_double), len(q),
                              _p(q, ctypes.c_double), _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle rho_q failed ({st})")
    return out[:, 0] + 1j * out[:, 1]


def structure_factor_q(pos, q, c=None) -> np.ndarray:
    """S(q) = |rho(q)|^2 / rho0 at arbitrary q (rho0 = sum c^2, N for unit strengths)."""
    pos = _pos(pos)
    rho0 = float(len(pos)) if c is None else float(np.sum(np.asarray(c, np.float64) ** 2))
    return np.abs(rho_q(pos, q, c)) ** 2 / rho0


def loss_grad_q(pos, q, W, S0, c=None, want_grad: bool = True):
    """Loss over arbitrary wave vectors (NUwNU): L = sum_k W_k (S(q_k) - S0_k)^2 and its
    position gradient.  Returns dict(S, loss, grad)."""
    pos = _pos(pos)
    N, d = pos.shape
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, d))
    K = len(q)
    W = np.ascontiguousarray(W, dtype=np.float64).ravel()
    S0 = np.ascontiguousarray(S0, dtype=np.float64).ravel()
    cc = None if c is None else _strengths(c, N)
    S = np.zeros(K)
    loss = np.zeros(1)
    grad = np.zeros((N, d)) if want_grad else None
    st = _load().oracle_loss_grad_q(d, N, _p(pos, ctypes.c_double), _p(cc, ctypes.c_double), K,
                                    _p(q, ctypes.c_double), _p(W, ctypes.c_double),
                                    _p(S0, ctypes.c_double), _p(S, ctypes.c_double),
                                    _p(loss, ctypes.c_double), _p(grad, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle loss_grad_q failed ({st})")
    return {"S": S, "loss": float(loss[0]), "grad": grad}


def grad_strengths_q(pos, q, W, S0, c) -> np.ndarray:
    """dL/dc_j of the loss over arbitrary wave vectors (Methods, Eq.
    lossweightgradient): the weights of fixed points, e.g. the pixels of a
    uniform grid (the UwNU variant)."""
    pos = _pos(pos)
    N, d = pos.shape
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, d))
    W = np.ascontiguousarray(W, dtype=np.float64).ravel()
    S0 = np.ascontiguousarray(S0, dtype=np.float64).ravel()
    cc = _strengths(c, N)
    out = np.zeros(N)
    st = _load().oracle_grad_c_q(d, N, _p(pos, ctypes.c_double), _p(cc, ctypes.c_double), len(q),
                                 _p(q, ctypes.c_double), _p(W, ctypes.c_double),
                                 _p(S0, ctypes.c_double), _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle grad_c_q failed ({st})")
    return out


def ewald_directions(d: int, e_inc, ns: int):
    """Scattered directions of the Ewald construction for the incident direction
    e_inc (a unit vector) and whether each lies in the forward half (main text,
    Eq. ewald; SI, single scattering): in 2D the ns - 1 directions at angles
    2 pi m / ns, m = 1 .. ns - 1, from e_inc (m = 0, the incident direction itself,
    is left out); in 3D an ns-point Fibonacci lattice on the sphere, z_i = 1 -
    (2i + 1)/ns, phi_i = i pi (3 - sqrt 5), in the frame whose z axis is e_inc
    (x axis: a x e_inc normalised, with a = e_z, or e_x when |e_inc . e_z| > 0.9).
    Forward: e_s . e_inc > 0 strictly, decided on the quadrature's integers so that
    the directions at exactly 90 degrees are not forward (2D: 4m < ns or 4m > 3ns;
    3D: z_i > 0, i.e. 2i + 1 < ns)."""
    e = np.asarray(e_inc, dtype=np.float64)
    if d == 2:
        m = np.arange(1, ns)
        th = np.arctan2(e[1], e[0]) + 2 * np.pi * m / ns
        es = np.stack([np.cos(th), np.sin(th)], 1)
        return es, (4 * m < ns) | (4 * m > 3 * ns)
    else:
        i = np.arange(ns)
        z = 1.0 - (2 * i + 1) / ns
        ph = i * np.pi * (3.0 - np.sqrt(5.0))
        rr = np.sqrt(1.0 - z * z)
        u = np.stack([rr * np.cos(ph), rr * np.sin(ph), z], 1)
        a = np.array([1.0, 0.0, 0.0]) if abs(e[2]) > 0.9 else np.array([0.0, 0.0, 1.0])
        e1 = np.cross(a, e)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(e, e1)
        es = u[:, :1] * e1 + u[:, 1:2] * e2 + u[:, 2:] * e
        return es, 2 * i + 1 < ns


def ewald_transmission(S_of_q, d: int, k: float, e_inc, ns: int) -> float:
    """T(k e_inc) = sum over forward scattered directions of S(q) / sum over all of
    them, q = k (e_s - e_inc) (Eq. ewald, the integrals by the quadrature of
    ewald_directions).  S_of_q: callable on [K][d] wave vectors."""
    es, fwd = ewald_directions(d, e_inc, ns)
    S = np.asarray(S_of_q(k * (es - np.asarray(e_inc, np.float64))), dtype=np.float64)
    return float(S[fwd].sum() / S.sum())


def pair_correlation(pos, L, M, xs) -> np.ndarray:
    """g(x) at the points xs [P][d] (Methods, pair correlation function
    optimisation): the periodic box turns the integral over k into a sum over the
    mode cube |n_a| <= M_a, n = 0 included,
        g(x) = Re[(1/N) sum_n (S(n) - 1) exp(-i k.x)] = (1/N) sum_n (S(n) - 1) cos(k.x)
    (unit strengths; S is even in k)."""
    pos = _pos(pos)
    N, d = pos.shape
    Lv = _box(L, d)
    modes = mode_vectors(d, M)
    S = structure_factor_cube(pos, L, M).ravel()
    k = 2 * np.pi * modes / Lv
    xs = np.asarray(xs, dtype=np.float64).reshape(-1, d)
    return np.cos(xs @ k.T) @ (S - 1.0) / N


def pair_correlation_loss_grad(pos, L, M, xs, wg, g0):
    """L_g = sum_x W_g (g - g0)^2 over the points xs and its position gradient
        dL_g/dr_j = sum_n gS(n) dS(n)/dr_j,   gS(n) = (1/N) sum_x 2 W_g (g - g0) cos(k.x)
    (the derivative of g in the Methods, written through the backward of S).
    Returns dict(loss, grad [N][d], g [P])."""
    pos = _pos(pos)
    N, d = pos.shape
    Lv = _box(L, d)
    modes = mode_vectors(d, M)
    k = 2 * np.pi * modes / Lv
    xs = np.asarray(xs, dtype=np.float64).reshape(-1, d)
    wg = np.asarray(wg, dtype=np.float64).ravel()
    g0 = np.asarray(g0, dtype=np.float64).ravel()
    C = np.cos(xs @ k.T)
    S = structure_factor_cube(pos, L, M).ravel()
    g = C @ (S - 1.0) / N
    r = g - g0
    gS = C.T @ (2.0 * wg * r) / N
    grad = sf_vjp(pos, L, modes, gS)
    return {"loss": float(np.sum(wg * r * r)), "grad": grad, "g": g}


def pair_finite_difference(pos, L, coords, h: float, sigma: float, eps: float = 1.0,
                           alpha: float = 2.0) -> np.ndarray:
    """(E(r_ja + h) - E(r_ja - h)) / 2h of the soft-core energy for coords [(j, a), ...],
    each from the differences of point j's own pairs (brute force, O(N) each)."""
    pos = _pos(pos)
    N, d = pos.shape
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, 2)
    cj = np.ascontiguousarray(coords[:, 0], dtype=np.int64)
    ca = np.ascontiguousarray(coords[:, 1], dtype=np.int32)
    out = np.zeros(len(coords))
    st = _load().oracle_pair_fd(d, N, _p(_box(L, d), ctypes.c_double), _p(pos, ctypes.c_double),
                                float(sigma), float(eps), float(alpha), len(coords),
                                _p(cj, ctypes.c_longlong), _p(ca, ctypes.c_int), float(h),
                                _p(out, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle pair finite difference failed ({st})")
    return out


def rho_direct(pos, L, modes, chunk: int = 100_000_000) -> np.ndarray:
    """rho(k) for a few listed modes by direct cos/sin of k.r_j (no per-point tables),
    for very many points; pos may be float32 (widened chunk by chunk, exactly)."""
    pos = np.asarray(pos)
    N, d = pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = modes.shape[0]
    total = np.zeros(2 * K)
    for s0 in range(0, N, chunk):
        part = np.ascontiguousarray(pos[s0:s0 + chunk], dtype=np.float64)
        out = np.zeros(2 * K)
        st = _load().oracle_rho_direct(d, part.shape[0], _p(_box(L, d), ctypes.c_double),
                                       _p(part, ctypes.c_double), K, _p(modes, ctypes.c_int),
                                       _p(out, ctypes.c_double))
        if st:
            raise RuntimeError(f"oracle_rho_direct failed ({st})")
        total += out
    return total[0::2] + 1j * total[1::2]


def loss_grad_from_rho(N: int, L, modes, W, S0, rho, grad_pos):
    """Loss, S and the gradient at the points grad_pos [G][d] from rho(k) on the
    listed modes (summed over N points, e.g. by rho_direct).  Returns dict(loss, S, grad)."""
    grad_pos = _pos(grad_pos)
    G, d = grad_pos.shape
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1, d)
    K = modes.shape[0]
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(K)
    S0 = np.ascontiguousarray(S0, dtype=np.float64).reshape(K)
    rh = np.ascontiguousarray(np.stack([np.real(rho), np.imag(rho)], 1), dtype=np.float64)
    S = np.zeros(K)
    loss = np.zeros(1)
    grad = np.zeros((G, d))
    st = _load().oracle_loss_grad_rho(d, int(N), _p(_box(L, d), ctypes.c_double), K,
                                      _p(modes, ctypes.c_int), _p(W, ctypes.c_double),
                                      _p(S0, ctypes.c_double), _p(rh, ctypes.c_double),
                                      _p(S, ctypes.c_double), _p(loss, ctypes.c_double), G,
                                      _p(grad_pos, ctypes.c_double), _p(grad, ctypes.c_double))
    if st:
        raise RuntimeError(f"oracle_loss_grad_rho failed ({st})")
    return {"loss": float(loss[0]), "S": S, "grad": grad}
