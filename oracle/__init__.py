"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and it
shares no code with it.  The numerical work is in ``oracle.c`` (plain loops in
double precision, see its header); this module only marshals numpy arrays and
writes out the two trivial reductions in numpy:

* the probed imaging condition of Eq. 3, image = scale * sum_i Ubar[i] * Vbar[i]
  (Section "Approximate gradient calculations"), and
* the misfit J = 1/2 sum (d - d_obs)^2 with residual res = d - d_obs.

``build()`` compiles ``oracle.c`` with gcc into ``liboracle.so`` beside it.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP, IEEE double: no fast-math, no FMA)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load(path: str):
    """Opens a compiled oracle library and declares its functions' signatures
    (``lib()`` caches the one built from ``oracle.c``)."""
    L = ctypes.CDLL(path)
    L.orc_forward.restype = ctypes.c_int
    L.orc_forward.argtypes = [
        ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_double,
        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
        _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
        ctypes.c_int, ctypes.c_long, _lp, _dp, _dp, _dp]
    L.orc_adjoint.restype = ctypes.c_int
    L.orc_adjoint.argtypes = [
        ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_double,
        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
        _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
        ctypes.c_long, _lp, _dp, _dp, _dp, _dp]
    L.orc_laplacian.restype = None
    L.orc_laplacian.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                ctypes.c_double, _dp, _dp]
    L.orc_damping_profile.restype = None
    L.orc_damping_profile.argtypes = [ctypes.c_long, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _dp]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_tti_apply.restype = None
    L.orc_tti_apply.argtypes = [ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_double,
                                _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.orc_tti_sweep.restype = ctypes.c_int
    L.orc_tti_sweep.argtypes = [
        ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_double,
        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
        _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp,
        ctypes.c_int, _dp, ctypes.c_long, _lp, _dp, _dp, _dp]
    for name in ("orc_sample_points", "orc_inject_points"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_int,
                      _dp, _dp, _dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load(_LIB)
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


@dataclasses.dataclass(frozen=True)
class Grid:
    ndim: int
    shape: tuple      # (nz, ny, nx), ny == 1 in 2D
    h: float
    dt: float
    nt: int
    nb: int
    c_ref: float
    R: float = 1e-3

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))

    @classmethod
    def of(cls, wl) -> "Grid":
        return cls(wl.ndim, tuple(wl.shape), wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R)


def _d(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def laplacian(ndim: int, u: np.ndarray, h: float) -> np.ndarray:
    """8th-order Laplacian of u[nz][ny][nx] (ny == 1 in 2D), zero outside."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    lib().orc_laplacian(ndim, nz, ny, nx, h, u.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def damping_profile(n: int, nb: int, h: float, c_ref: float, R: float) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().orc_damping_profile(n, nb, h, c_ref, R, out.ctypes.data_as(_dp))
    return out


def sample_points(ndim: int, field: np.ndarray, pos) -> np.ndarray:
    """Pr: multilinear interpolation of field [nz][ny][nx] at positions [n][3]
    (z, y, x) in grid units."""
    f = np.ascontiguousarray(field, dtype=np.float64)
    nz, ny, nx = f.shape
    p, pp = _d(np.reshape(pos, (-1, 3)))
    out = np.zeros(p.shape[0])
    rc = lib().orc_sample_points(ndim, nz, ny, nx, p.shape[0], pp, f.ctypes.data_as(_dp),
                                 out.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError(f"oracle sampling rejected its input (code {rc})")
    return out


def inject_points(ndim: int, shape, pos, val) -> np.ndarray:
    """Ps^T: a zero field [nz][ny][nx] with val[p] spread onto the corners of
    position p by the multilinear weights."""
    nz, ny, nx = shape
    f = np.zeros((nz, ny, nx))
    p, pp = _d(np.reshape(pos, (-1, 3)))
    v, vp = _d(np.ravel(val))
    assert v.size == p.shape[0]
    rc = lib().orc_inject_points(ndim, nz, ny, nx, p.shape[0], pp, vp, f.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError(f"oracle injection rejected its input (code {rc})")
    return f


def forward(g: Grid, m, src_pos, q, rec_pos, Z=None, what: str = "utt", sample_idx=None,
            hist: bool = False, final: bool = False, want_d: bool = True) -> dict:
    """Forward sweep.  Returns dict with d [nt][nrec], Ubar [r][M] (if Z given),
    hist [nt][N] (if hist), final [2][N] = (u^nt, u^{nt-1}) (if final)."""
    nz, ny, nx = g.shape
    N = g.N
    m, mp = _d(np.ravel(m))
    src, sp = _d(np.reshape(src_pos, (-1, 3)))
    q, qp = _d(np.reshape(q, (g.nt, -1)))
    rec, rp = _d(np.reshape(rec_pos, (-1, 3)))
    assert m.size == N and q.shape[1] == src.shape[0]
    out = {}
    d = np.zeros((g.nt, rec.shape[0])) if want_d else None
    r = 0
    zp = up = None
    sidx = None
    M = N
    if Z is not None:
        Zd, zp = _d(Z)
        r = Zd.shape[1]
        assert Zd.shape[0] == g.nt
        if sample_idx is not None:
            sidx = np.ascontiguousarray(sample_idx, dtype=np.int64)
            M = sidx.size
        Ub = np.zeros((r, M))
        up = Ub.ctypes.data_as(_dp)
        out["Ubar"] = Ub
    H = np.zeros((g.nt, N)) if hist else None
    F = np.zeros((2, N)) if final else None
    rc = lib().orc_forward(
        g.ndim, nz, ny, nx, g.h, g.dt, g.nt, g.nb, g.c_ref, g.R, mp, src.shape[0], sp, qp,
        rec.shape[0], rp, d.ctypes.data_as(_dp) if d is not None else None, r, zp,
        1 if what == "utt" else 0, M if sidx is not None else 0,
        sidx.ctypes.data_as(_lp) if sidx is not None else None, up,
        H.ctypes.data_as(_dp) if H is not None else None,
        F.ctypes.data_as(_dp) if F is not None else None)
    if rc != 0:
        raise ValueError(f"oracle forward rejected its input (code {rc})")
    if d is not None:
        out["d"] = d
    if H is not None:
        out["hist"] = H
    if F is not None:
        out["final"] = F
    return out


def adjoint(g: Grid, m, rec_pos, res, src_pos=None, Z=None, sample_idx=None,
            fwd_hist=None, lam_hist: bool = False) -> dict:
    """Adjoint sweep driven by res [nt][nrec].  Returns dict with qadj
    [nt][nsrc] (if src_pos), Vbar [r][M] (if Z), corr [N] = sum_n fwd_hist[n]
    * lam^n (if fwd_hist), hist [nt][N] (if lam_hist)."""
    nz, ny, nx = g.shape
    N = g.N
    m, mp = _d(np.ravel(m))
    rec, rp = _d(np.reshape(rec_pos, (-1, 3)))
    res, resp = _d(np.reshape(res, (g.nt, -1)))
    assert res.shape[1] == rec.shape[0]
    out = {}
    nsrc = 0
    sp = qa = None
    if src_pos is not None:
        src, sp = _d(np.reshape(src_pos, (-1, 3)))
        nsrc = src.shape[0]
        qa = np.zeros((g.nt, nsrc))
        out["qadj"] = qa
    r = 0
    zp = vp = None
    sidx = None
    M = N
    if Z is not None:
        Zd, zp = _d(Z)
        r = Zd.shape[1]
        if sample_idx is not None:
            sidx = np.ascontiguousarray(sample_idx, dtype=np.int64)
            M = sidx.size
        Vb = np.zeros((r, M))
        vp = Vb.ctypes.data_as(_dp)
        out["Vbar"] = Vb
    fh = fhp = corr = None
    if fwd_hist is not None:
        fh, fhp = _d(fwd_hist)
        corr = np.zeros(N)
        out["corr"] = corr
    H = np.zeros((g.nt, N)) if lam_hist else None
    rc = lib().orc_adjoint(
        g.ndim, nz, ny, nx, g.h, g.dt, g.nt, g.nb, g.c_ref, g.R, mp, rec.shape[0], rp, resp,
        nsrc, sp, qa.ctypes.data_as(_dp) if qa is not None else None, r, zp,
        M if sidx is not None else 0, sidx.ctypes.data_as(_lp) if sidx is not None else None,
        vp, fhp, corr.ctypes.data_as(_dp) if corr is not None else None,
        H.ctypes.data_as(_dp) if H is not None else None)
    if rc != 0:
        raise ValueError(f"oracle adjoint rejected its input (code {rc})")
    if H is not None:
        out["hist"] = H
    return out


def image(Ubar: np.ndarray, Vbar: np.ndarray, scale: float) -> np.ndarray:
    """Eq. 3: scale * sum over probes of Ubar[i] * Vbar[i] (per cell)."""
    return scale * (np.asarray(Ubar, np.float64) * np.asarray(Vbar, np.float64)).sum(axis=0)


def misfit(d: np.ndarray, d_obs: np.ndarray):
    res = np.asarray(d, np.float64) - np.asarray(d_obs, np.float64)
    return 0.5 * float((res * res).sum()), res


def exact_gradient(g: Grid, m, src_pos, q, rec_pos, d_obs):
    """Eq. 2 with the full history: J and g = -sum_n (d2u/dt2)^n * lam^n."""
    f = forward(g, m, src_pos, q, rec_pos, what="utt", hist=True)
    J, res = misfit(f["d"], d_obs)
    a = adjoint(g, m, rec_pos, res, fwd_hist=f["hist"])
    return J, -a["corr"]


def probed_gradient(g: Grid, m, src_pos, q, rec_pos, d_obs, Z, sample_idx=None):
    """Eq. 3: J and g_r = -(1/r) sum_i Ubar[i] * Vbar[i], Ubar probing d2u/dt2."""
    f = forward(g, m, src_pos, q, rec_pos, Z=Z, what="utt", sample_idx=sample_idx)
    J, res = misfit(f["d"], d_obs)
    a = adjoint(g, m, rec_pos, res, Z=Z, sample_idx=sample_idx)
    r = np.shape(Z)[1]
    return J, image(f["Ubar"], a["Vbar"], -1.0 / r), f, a


# ---------------------------------------------------------------------------
# pseudo-acoustic TTI (coupled p, q); see the header of oracle.c
# ---------------------------------------------------------------------------
def stacked_probed_gradient(g: Grid, m, shots, Zs):
    """The stack over sources (the sum over shots of each shot's probed
    gradient, Eq. 3, every shot with its own probe matrix; Section
    "Approximate gradient calculations", the remark after Eq. 4 on noise that
    stacks out over sources).  shots: (src_pos, q, rec_pos, d_obs) per shot,
    Zs: the matching probe matrices.  Returns (sum of misfits, summed
    gradient)."""
    J, G = 0.0, np.zeros(g.N)
    for (src_pos, q, rec_pos, d_obs), Z in zip(shots, Zs):
        Ji, gi, _, _ = probed_gradient(g, m, src_pos, q, rec_pos, d_obs, Z)
        J += Ji
        G += gi
    return J, G


def tti_apply(eps, delta, theta, phi, p, q, h, transpose=False):
    """The TTI spatial operator (or its transpose) on fields [nz][ny][nx]."""
    p = np.ascontiguousarray(p, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    nz, ny, nx = p.shape
    a = [np.ascontiguousarray(np.broadcast_to(v, p.shape), np.float64)
         for v in (eps, delta, theta, phi)]
    op, oq = np.empty_like(p), np.empty_like(p)
    lib().orc_tti_apply(nz, ny, nx, h, *(x.ctypes.data_as(_dp) for x in a), int(transpose),
                        p.ctypes.data_as(_dp), q.ctypes.data_as(_dp), op.ctypes.data_as(_dp),
                        oq.ctypes.data_as(_dp))
    return op, oq


def _tti_sweep(adjoint, g: Grid, m, aniso, inj_pos, inj_val, smp_pos, Z=None, hist=None,
               want_hist=False, sample_idx=None):
    nz, ny, nx = g.shape
    N = g.N
    m, mp = _d(np.ravel(m))
    an = [_d(np.ravel(x)) for x in aniso]          # eps, delta, theta, phi
    ip, ipp = _d(np.reshape(inj_pos, (-1, 3)))
    iv, ivp = _d(np.reshape(inj_val, (g.nt, -1)))
    out = {}
    smp = sp = None
    nsmp = 0
    if smp_pos is not None:
        sp_arr, spp = _d(np.reshape(smp_pos, (-1, 3)))
        nsmp = sp_arr.shape[0]
        smp = np.zeros((g.nt, nsmp))
        sp = spp
        out["d" if not adjoint else "qadj"] = smp
    r = 0
    zp = up = None
    sidx = None
    if Z is not None:
        Zd, zp = _d(Z)
        r = Zd.shape[1]
        M = N
        if sample_idx is not None:
            sidx = np.ascontiguousarray(sample_idx, dtype=np.int64)
            M = sidx.size
        Ub = np.zeros((2, r, M))
        up = Ub.ctypes.data_as(_dp)
        out["bar"] = Ub
    fh = corr = None
    if not adjoint and want_hist:
        fh = np.zeros((2, g.nt, N))
        out["hist"] = fh
    if adjoint and hist is not None:
        fh = np.ascontiguousarray(hist, np.float64)
        corr = np.zeros(N)
        out["corr"] = corr
    rc = lib().orc_tti_sweep(
        int(adjoint), nz, ny, nx, g.h, g.dt, g.nt, g.nb, g.c_ref, g.R, mp,
        *(x[1] for x in an), ip.shape[0], ipp, ivp, nsmp, sp,
        smp.ctypes.data_as(_dp) if smp is not None else None, r, zp,
        sidx.size if sidx is not None else 0,
        sidx.ctypes.data_as(_lp) if sidx is not None else None, up,
        fh.ctypes.data_as(_dp) if fh is not None else None,
        corr.ctypes.data_as(_dp) if corr is not None else None)
    if rc != 0:
        raise ValueError(f"oracle TTI sweep rejected its input (code {rc})")
    return out


def tti_forward(g: Grid, m, aniso, src_pos, q, rec_pos, Z=None, hist=False, sample_idx=None):
    """d [nt][nrec] = p at the receivers; bar [2][r][M] = Z^T (p_tt, q_tt) on
    the cells sample_idx (all N cells when None)."""
    return _tti_sweep(False, g, m, aniso, src_pos, q, rec_pos, Z=Z, want_hist=hist,
                      sample_idx=sample_idx)


def tti_adjoint(g: Grid, m, aniso, rec_pos, res, src_pos=None, Z=None, fwd_hist=None,
                sample_idx=None):
    """bar [2][r][M] = Z^T (lam_p, lam_q); qadj = Ps (lam_p + lam_q); corr."""
    return _tti_sweep(True, g, m, aniso, rec_pos, res, src_pos, Z=Z, hist=fwd_hist,
                      sample_idx=sample_idx)


def tti_exact_gradient(g: Grid, m, aniso, src_pos, q, rec_pos, d_obs):
    f = tti_forward(g, m, aniso, src_pos, q, rec_pos, hist=True)
    J, res = misfit(f["d"], d_obs)
    a = tti_adjoint(g, m, aniso, rec_pos, res, fwd_hist=f["hist"])
    return J, -a["corr"]


def tti_probed_gradient(g: Grid, m, aniso, src_pos, q, rec_pos, d_obs, Z, sample_idx=None):
    f = tti_forward(g, m, aniso, src_pos, q, rec_pos, Z=Z, sample_idx=sample_idx)
    J, res = misfit(f["d"], d_obs)
    a = tti_adjoint(g, m, aniso, rec_pos, res, Z=Z, sample_idx=sample_idx)
    r = np.shape(Z)[1]
    img = image(f["bar"][0], a["bar"][0], -1.0 / r) + image(f["bar"][1], a["bar"][1], -1.0 / r)
    return J, img, f, a


# ---------------------------------------------------------------------------
# range-finder probes (Section "Randomized trace estimation": probing vectors
# Q from a partial QR factorization of A Z, Z a Rademacher +-1 matrix).  A is
# read as the forward history H [nt][N] of u_tt, sketched in space: Y = H Omega
# with Omega [N][r] Rademacher, Q = qr(Y), then Eq. 3 with Z = Q and scale 1
# (Q Q^T is an orthogonal projector, no 1/r).
# ---------------------------------------------------------------------------
def sketch_signs(N: int, r: int, seed: int) -> np.ndarray:
    """Omega [N][r]: entry (x, i) = 1 - 2 b with b the bit i % 64 of word i // 64
    of the Philox4x64-10 block (key (seed, 0)) at counter (x + 1, 0, 0, 0).
    numpy's Philox increments its counter before each block, so a generator
    started at counter 0 yields exactly the blocks of cells 0, 1, 2, ..."""
    assert 0 < r <= 256
    bg = np.random.Philox(counter=[0, 0, 0, 0], key=[int(seed), 0])
    w = bg.random_raw(4 * N).reshape(N, 4)
    i = np.arange(r)
    bits = (w[:, i // 64] >> (i % 64).astype(np.uint64)) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def sketch(g: Grid, m, src_pos, q, seed: int, r: int) -> np.ndarray:
    """Y [nt][r] = H Omega, H [nt][N] the forward history of u_tt."""
    rec = np.zeros((1, 3))
    f = forward(g, m, src_pos, q, rec, what="utt", hist=True, want_d=False)
    return f["hist"] @ sketch_signs(g.N, r, seed)


def range_finder(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis [nt][r] of the column space of Y (Householder QR)."""
    Q, _ = np.linalg.qr(np.asarray(Y, np.float64))
    return Q


def rf_gradient(g: Grid, m, src_pos, q, rec_pos, d_obs, seed: int, r: int):
    """J and g = -sum_i Ubar[i] * Vbar[i] with Z = Q = range_finder(sketch)."""
    Y = sketch(g, m, src_pos, q, seed, r)
    Q = range_finder(Y)
    f = forward(g, m, src_pos, q, rec_pos, Z=Q, what="utt")
    J, res = misfit(f["d"], d_obs)
    a = adjoint(g, m, rec_pos, res, Z=Q)
    return J, image(f["Ubar"], a["Vbar"], -1.0), Q, Y


# ---------------------------------------------------------------------------
# subsurface-offset image volume (Eq. 4)
# ---------------------------------------------------------------------------
def offset_gathers(Ubar, Vbar, shape, nh: int, scale: float) -> np.ndarray:
    """G [2 nh + 1][N]: G[h + nh][x] = scale * sum_i Ubar[i][x + h] Vbar[i][x - h]
    with the offset h along x (the last axis), zero where x + h or x - h leaves
    the row.  Ubar, Vbar are [r][N] (rows)."""
    nz, ny, nx = shape
    U = np.asarray(Ubar, np.float64).reshape(-1, nz, ny, nx)
    V = np.asarray(Vbar, np.float64).reshape(-1, nz, ny, nx)
    G = np.zeros((2 * nh + 1, nz, ny, nx))
    for h in range(-nh, nh + 1):
        for x in range(nx):
            xu, xv = x + h, x - h
            if 0 <= xu < nx and 0 <= xv < nx:
                G[h + nh, :, :, x] = (U[:, :, :, xu] * V[:, :, :, xv]).sum(axis=0)
    return scale * G.reshape(2 * nh + 1, -1)
