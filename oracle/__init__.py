"""ctypes front end of the plain FP64 CPU oracle (``nlte_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the benchmark's
CPU-baseline leg are its only users.  The HIP library never imports or links it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlte_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE order, no contraction, OpenMP over points)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_species.argtypes = [C.c_void_p, C.c_int, _dp, _dp, C.c_double, C.c_int, _ip, _ip,
                                     _dp, C.c_int, _ip, _ip, C.c_int, _dp, _dp]
        L.or_set_model.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int, _ip,
                                   C.c_void_p]
        L.or_set_rays.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_set_quadrature.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.or_set_params.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int]
        L.or_n_pairs.argtypes = [C.c_void_p]
        L.or_line_width_speed.argtypes = [C.c_void_p, _dp]
        L.or_planck.argtypes = [C.c_double, C.c_double]
        L.or_planck.restype = C.c_double
        L.or_coll_rates.argtypes = [C.c_void_p, C.c_int64, _dp, _dp]
        L.or_lte.argtypes = [C.c_void_p, _dp]
        L.or_walk.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.or_pair_nodes.argtypes = [C.c_void_p, _dp, C.c_int64, C.c_int, C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int)]
        L.or_solve_ray.argtypes = [C.c_int, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                   C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.c_void_p]
        L.or_formal_solve.argtypes = [C.c_void_p, _dp, C.c_int64, C.c_void_p, _dp, _dp, _dp]
        L.or_stateq.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.c_void_p]
        L.or_rel_change.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_double)]
        L.or_rel_change.restype = C.c_double
        L.or_run_ali.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_int, C.c_double, _dp]
        L.or_walk_all.argtypes = [C.c_void_p, _lp, C.c_void_p]
        L.or_walk_all.restype = C.c_int64
        L.or_features.argtypes = [C.c_void_p, _dp]
        L.or_formal_solve_band.argtypes = [C.c_void_p, _dp, C.c_int64, C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_solve_ray_gen.argtypes = [C.c_int, _dp, _dp, C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                       C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_solve_ray_gen.restype = C.c_int
        L.or_formal_solve_scat.argtypes = [C.c_void_p, _dp, _dp, C.c_void_p, _dp, C.c_int64, C.c_void_p, _dp, _dp,
                                           _dp, _dp]
        L.or_formal_solve_scat.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int) -> None:
    """Threads of the oracle's loops over origin points."""
    lib().or_set_threads(int(n))


def planck(nu: float, T: float) -> float:
    return lib().or_planck(nu, T)


def solve_ray(z, chi, S, I_lo, I_hi, o, tau_floor=1e-100, want_all=False):
    """One Feautrier solve on explicit nodes: returns (u_o, Lambda_oo, ueff_o[, u_all])."""
    z, chi, S = _f64(z), _f64(chi), _f64(S)
    N = z.shape[0]
    u, lam, ue = C.c_double(), C.c_double(), C.c_double()
    ua = np.zeros(N) if want_all else None
    lib().or_solve_ray(N, z, chi, S, I_lo, I_hi, int(o), tau_floor, C.byref(u), C.byref(lam),
                       C.byref(ue), ua.ctypes.data if want_all else None)
    if want_all:
        return u.value, lam.value, ue.value, ua
    return u.value, lam.value, ue.value


def solve_ray_gen(z, chi, Splus, sigma, I_lo, I_hi, o, own=0.0, tau_floor=1e-100, chim=None):
    """Generalised Feautrier solve (both equations of Eq. GFE) on explicit nodes with total
    opacity chi = chi + chi^+ and, optionally, the odd scattering opacity chim = chi^- along
    +z: returns (u_o, Lambda_oo, ueff_o, v_o)."""
    z, chi, Splus, sigma = _f64(z), _f64(chi), _f64(Splus), _f64(sigma)
    cm = None if chim is None else _f64(chim)
    u, lam, ue, v = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    rc = lib().or_solve_ray_gen(z.shape[0], z, chi, None if cm is None else cm.ctypes.data, Splus, sigma,
                                I_lo, I_hi, int(o), tau_floor, own, C.byref(u), C.byref(lam), C.byref(ue),
                                C.byref(v))
    if rc != 0:
        raise ValueError("the integrating factor e^M leaves the FP64 range (|M| > 700)")
    return u.value, lam.value, ue.value, v.value


class Oracle:
    """One model + species + rays + quadrature, as the oracle sees it."""

    def __init__(self, model, species, rays, quad_x, quad_w, t_cmb=2.725, f_sub=0.25,
                 tau_floor=1e-100, use_alo=True):
        L = lib()
        self._L = L
        self.c = L.or_create()
        sp = species
        self.species = sp
        self.n_lev = sp.n_lev
        self.n_lines = sp.n_lines
        self._keep = []
        L.or_set_species(self.c, sp.n_lev, _f64(sp.energy), _f64(sp.weight), float(sp.mass),
                         sp.n_lines, _i32(sp.line_up), _i32(sp.line_lo), _f64(sp.line_A),
                         int(sp.coll_up.shape[0]), _i32(sp.coll_up), _i32(sp.coll_lo),
                         int(sp.coll_T.shape[0]), _f64(sp.coll_T), _f64(sp.coll_K))
        m = model
        self.P = m.n_points
        bnd = None
        if m.boundary is not None:
            bnd = np.ascontiguousarray(m.boundary, dtype=np.uint8)
            self._keep.append(bnd)
        L.or_set_model(self.c, self.P, _f64(m.pos), _f64(m.vel), _f64(m.n_h2), _f64(m.temperature),
                       _f64(m.v_turb), _f64(m.abundance), int(m.nbr.shape[1]), _i32(m.nbr),
                       bnd.ctypes.data if bnd is not None else None)
        npairs = L.or_set_rays(self.c, int(rays.shape[0]), _f64(rays))
        if npairs < 0:
            raise ValueError("ray set is not point-symmetric")
        self.n_rays = int(rays.shape[0])
        self.n_pairs = npairs
        self.rays = np.array(rays, dtype=np.float64)
        self.model = model
        self.t_cmb = t_cmb
        self.tau_floor = tau_floor
        L.or_set_quadrature(self.c, int(quad_x.shape[0]), _f64(quad_x), _f64(quad_w))
        self.n_q = int(quad_x.shape[0])
        L.or_set_params(self.c, t_cmb, f_sub, tau_floor, 1 if use_alo else 0)

    def __del__(self):
        try:
            self._L.or_destroy(self.c)
        except Exception:
            pass

    def line_width_speed(self):
        out = np.zeros(self.P)
        self._L.or_line_width_speed(self.c, out)
        return out

    def coll_rates(self, p):
        n = int(self.species.coll_up.shape[0])
        a, b = np.zeros(n), np.zeros(n)
        self._L.or_coll_rates(self.c, int(p), a, b)
        return a, b

    def lte(self):
        out = np.zeros((self.P, self.n_lev))
        self._L.or_lte(self.c, out)
        return out

    def walk(self, O, ray):
        n = self._L.or_walk(self.c, int(O), int(ray), None, None, 0)
        cells = np.zeros(max(n, 1), dtype=np.int32)
        Z = np.zeros(max(n, 1))
        self._L.or_walk(self.c, int(O), int(ray), cells.ctypes.data, Z.ctypes.data, n)
        return cells[:n].copy(), Z[:n].copy()

    def walk_all(self):
        """CSR of every (point, ray) walk: (offsets [P*n_rays+1], cells)."""
        off = np.zeros(self.P * self.n_rays + 1, dtype=np.int64)
        tot = self._L.or_walk_all(self.c, off, None)
        cells = np.zeros(max(tot, 1), dtype=np.int32)
        self._L.or_walk_all(self.c, off, cells.ctypes.data)
        return off, cells[:tot]

    def features(self):
        """Warm-start surrogate inputs [P][8] (raw, unstandardised)."""
        out = np.zeros((self.P, 8))
        self._L.or_features(self.c, out)
        return out

    def pair_nodes(self, pops, O, pair):
        pops = _f64(pops)
        io = C.c_int()
        N = self._L.or_pair_nodes(self.c, pops, int(O), int(pair), 0, None, None, None, None, None,
                                  C.byref(io))
        z, a, b = np.zeros(N), np.zeros(N), np.zeros(N)
        kap, S = np.zeros((N, self.n_lines)), np.zeros((N, self.n_lines))
        self._L.or_pair_nodes(self.c, pops, int(O), int(pair), N, z.ctypes.data, a.ctypes.data,
                              b.ctypes.data, kap.ctypes.data, S.ctypes.data, C.byref(io))
        return dict(z=z, a=a, b=b, kappa=kap, S=S, o=io.value)

    def formal_solve(self, pops, sel=None):
        pops = _f64(pops)
        if sel is None:
            n = self.P
            selp = None
            sel_arr = None
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            n = sel_arr.shape[0]
            selp = sel_arr.ctypes.data
        J = np.zeros((n, self.n_lines))
        Je = np.zeros((n, self.n_lines))
        Ls = np.zeros((n, self.n_lines))
        self._L.or_formal_solve(self.c, pops, n, selp, J, Je, Ls)
        return J, Je, Ls

    def formal_solve_band(self, pops, sel=None):
        """Band ALO of width one node: J, Jeff, L as formal_solve, plus Jb (J without the
        band's share), Ld (diagonal with the neighbours' interpolated part) and Ln
        [n][n_lines][n_rays] (coupling to the first cell of the walk along each ray)."""
        pops = _f64(pops)
        if sel is None:
            n, selp = self.P, None
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            n, selp = sel_arr.shape[0], sel_arr.ctypes.data
        out = [np.zeros((n, self.n_lines)) for _ in range(5)]
        Ln = np.zeros((n, self.n_lines, self.n_rays))
        self._L.or_formal_solve_band(self.c, pops, n, selp, *out, Ln)
        return (*out, Ln)

    def line_frequencies(self):
        sp = self.species
        return (sp.energy[sp.line_up] - sp.energy[sp.line_lo]) / 6.62607015e-27

    def scattering_start(self):
        """Initial J_nu [P][n_lines][n_q] of the scattering iteration: the boundary
        intensity (CMB at each line's centre) everywhere."""
        Ib = np.array([planck(nu, self.t_cmb) for nu in self.line_frequencies()])
        return np.broadcast_to(Ib[None, :, None], (self.P, self.n_lines, self.n_q)).copy()

    def formal_solve_scat(self, pops, chi_sca, Jnu_in, sel=None, chi_dip=None):
        """Formal solve with coherent scattering of opacity chi_sca + chi_dip . n
        (chi_sca [P][n_lines], chi_dip [P][n_lines][3] or None; cm^-1) driven by the previous
        weighted mean intensity Jw (J_nu for chi_dip = None): returns (J, Jeff, L,
        Jw_out [n][n_lines][n_q])."""
        pops = _f64(pops)
        if sel is None:
            n, selp = self.P, None
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            n, selp = sel_arr.shape[0], sel_arr.ctypes.data
        J, Je, Ls = (np.zeros((n, self.n_lines)) for _ in range(3))
        Jnu = np.zeros((n, self.n_lines, self.n_q))
        dip = None if chi_dip is None else _f64(chi_dip)
        rc = self._L.or_formal_solve_scat(self.c, pops, _f64(chi_sca), None if dip is None else dip.ctypes.data,
                                          _f64(Jnu_in), n, selp, J, Je, Ls, Jnu)
        if rc == -1:
            raise ValueError("the scattering solve needs an ascending quadrature")
        if rc == -3:
            raise ValueError("|chi_dip| exceeds chi_sca: a negative scattering opacity")
        if rc == -2:
            raise ValueError("a ray's integrating factor e^M leaves the FP64 range (|M| > 700)")
        return J, Je, Ls, Jnu

    def run_ali_scat(self, chi_sca, pops_init=None, max_iter=50, tol=1e-4, chi_dip=None):
        """ALI with scattering: each iteration one formal solve driven by the previous J_nu
        (starting from scattering_start()), then the statistical equilibrium.  Returns
        (populations, changes, last J_nu)."""
        pops = self.lte() if pops_init is None else _f64(pops_init).copy()
        Jnu = self.scattering_start()
        ch = []
        for _ in range(max_iter):
            J, Je, Ls, Jnu = self.formal_solve_scat(pops, chi_sca, Jnu, chi_dip=chi_dip)
            new, _ = self.stateq(pops, J, Je, Ls)
            ch.append(self.rel_change(pops, new)[0])
            pops = new
            if ch[-1] < tol:
                break
        return pops, np.array(ch), Jnu

    def stateq(self, pops_old, J, Jeff, L):
        out = np.zeros((self.P, self.n_lev))
        flags = np.zeros(self.P, dtype=np.uint8)
        self._L.or_stateq(self.c, _f64(pops_old), _f64(J), _f64(Jeff), _f64(L), out,
                          flags.ctypes.data)
        return out, flags

    def image(self, pops, ray, line, v_ch, points=None):
        """Sec. 3.5: intensity leaving the model along direction `ray` at the far end of the
        ray pair through every point, at observer-frame channel velocities v_ch [cm/s] of
        line `line` (profile offset x = (v - n.v_k)/v_w,k at node k), with CMB intensity
        entering at both ends: I_out = 2 u_end - I_in from the pair's second-order
        solution.  Returns I [P][n_ch] (rows of `points` only, if given) and the
        image-plane coordinates [P][2]."""
        pops = _f64(pops)
        v_ch = np.atleast_1d(np.asarray(v_ch, dtype=np.float64))
        dirs = self.rays
        n = dirs[ray]
        # the pair holding this ray, and whether it is the pair's representative
        pair, forward = None, None
        for p in range(self.n_pairs):
            r = self._pair_rep(p)
            if r == ray:
                pair, forward = p, True
            elif np.allclose(dirs[r], -n, atol=1e-12):
                pair, forward = p, False
        sp = self.species
        nu = (sp.energy[sp.line_up[line]] - sp.energy[sp.line_lo[line]]) / 6.62607015e-27
        I_in = planck(nu, self.t_cmb)
        vw = self.line_width_speed()
        vel = self.model.vel
        pts = range(self.P) if points is None else [int(p) for p in points]
        out = np.zeros((len(pts), v_ch.shape[0]))
        for row, O in enumerate(pts):
            nd = self.pair_nodes(pops, O, pair)
            z, a, b = nd["z"], nd["a"], nd["b"]
            kap, S = nd["kappa"][:, line], nd["S"][:, line]
            # frame of O: x_k = a_k x_O - b_k along the representative's direction m;
            # for the antipode the propagation direction is -m and x_k = a_k x_O + b_k
            nvO = float(np.dot(n, vel[O]))
            for c, v in enumerate(v_ch):
                xO = (v - nvO) / vw[O]
                x = a * xO - b if forward else a * xO + b
                chi = kap * np.exp(-x * x)
                _, _, _, u = solve_ray(z, chi, S, I_in, I_in, nd["o"], tau_floor=self.tau_floor, want_all=True)
                u_end = u[-1] if forward else u[0]
                out[row, c] = 2.0 * u_end - I_in
        return out, image_plane(self.model.pos, n)

    def _pair_rep(self, p):
        """Representative ray of pair p (the lower index of the two antipodes)."""
        reps = [r for r in range(self.n_rays)
                if r == min(r, int(np.argmin(np.linalg.norm(self.rays + self.rays[r], axis=1))))]
        return reps[p]

    def rel_change(self, old, new):
        mean = C.c_double()
        mx = self._L.or_rel_change(self.c, _f64(old), _f64(new), C.byref(mean))
        return mx, mean.value

    def run_ali(self, pops_init=None, max_iter=50, tol=1e-4):
        out = np.zeros((self.P, self.n_lev))
        ch = np.zeros(max_iter)
        pi = None
        if pops_init is not None:
            pi = _f64(pops_init)
        it = self._L.or_run_ali(self.c, pi.ctypes.data if pi is not None else None, out, max_iter, tol, ch)
        return out, ch[:it].copy()


def from_workload(w, **kw) -> Oracle:
    return Oracle(w.model, w.species, w.rays, w.quad_x, w.quad_w, t_cmb=w.t_cmb, f_sub=w.f_sub, **kw)


def image_plane(pos, n):
    """Coordinates of points on the plane orthogonal to direction n: (x . e1, x . e2) with
    e1 = (z x n)/|z x n| (x-axis instead of z when |n_z| > 0.9) and e2 = n x e1."""
    n = np.asarray(n, dtype=np.float64)
    ref = np.array([0.0, 0.0, 1.0]) if abs(n[2]) <= 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(ref, n)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    pos = np.asarray(pos, dtype=np.float64)
    return np.stack([pos @ e1, pos @ e2], axis=1)


def morton_order(pos, offsets=None):
    """Processing order of the points: within each model (offsets, default one model), by
    the Morton code of coordinates quantised to 21 bits over the model's bounding box,
    q = floor((x - min) / (max - min) * (2^21 - 1)) (0 for a flat extent), bits
    interleaved x, y, z from the most significant; equal codes keep index order."""
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    offsets = [0, P] if offsets is None else list(offsets)
    order = np.empty(P, dtype=np.int64)
    for m in range(len(offsets) - 1):
        a, b = int(offsets[m]), int(offsets[m + 1])
        x = pos[a:b]
        lo, hi = x.min(axis=0), x.max(axis=0)
        q = np.zeros((b - a, 3), dtype=np.uint64)
        for d in range(3):
            ext = hi[d] - lo[d]
            if ext > 0:
                q[:, d] = np.floor((x[:, d] - lo[d]) / ext * 2097151.0).astype(np.uint64)
        code = np.zeros(b - a, dtype=np.uint64)
        for bit in range(21):
            for d in range(3):
                code |= ((q[:, d] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + 2 - d)
        order[a:b] = a + np.argsort(code, kind="stable")
    return order
