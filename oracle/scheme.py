"""The six coupled LBM schemes, one plain FP64 time step at a time
(test infrastructure, see oracle/__init__.py).

Populations are held post-streaming: ``f(x, t, q)``.  One call of ``step``
takes the moments of all six sets at time t, builds the sources, the forces
and the post-collision sets exactly in the order the paper describes them, and
streams them to t + 1, applying the boundary rules of Sec. 3.5 (Tables 1-2,
Eqs. (159)-(164)).  Nothing is fused or reordered for speed.

Where the paper leaves a choice open, the reading taken is stated next to the
line that makes it, under a short id (R1..R17) that the tests also use.
"""
import math

import numpy as np

from . import equilibria as eq
from .lattice import CS2, by_name

SCHEMES = ("g", "l", "ag", "al", "bg", "bl")
FACE_AXES = {"x": 0, "y": 1, "z": 2}


def _ramp(t, ymax, ymin, n_t):
    """Inlet ramp, Eq. (153): (ymax - ymin) tanh(t / n_t) + ymin."""
    if n_t is None or n_t <= 0:
        return ymax
    return (ymax - ymin) * math.tanh(t / n_t) + ymin


def spalding_B(x):
    """B(x) = x H(x) H(1-x) + H(x-1) of Eq. (93).

    Reading R2: H(0) = 1/2 (the half-maximum convention), with which B is the
    clamp of x to [0, 1] at every x, including x = 0 and x = 1.
    """
    H = lambda s: np.heaviside(s, 0.5)
    return x * H(x) * H(1.0 - x) + H(x - 1.0)


class Params:
    """Scheme parameters in lattice units (hat quantities)."""

    def __init__(self, cfg):
        self.lat = by_name(cfg["lattice"])
        D = self.lat.D
        self.shape = tuple(int(cfg[k]) for k in ("nz", "ny", "nx")[3 - D:])   # C order, x fastest
        bc = cfg.get("bc", {})
        self.bc = {}
        for name in "xyz"[:D]:
            for side in "-+":
                self.bc[name + side] = bc.get(name + side, "periodic")
            assert (self.bc[name + "-"] == "periodic") == (self.bc[name + "+"] == "periodic"), \
                "periodic faces come in pairs"
        self.up_axis = int(cfg.get("up_axis", D - 1))
        self.rho_g = float(cfg["rho_g"])
        self.rho_l = float(cfg["rho_l"])
        self.R = self.rho_l / self.rho_g                      # R = rho_l / rho_g, text after Eq. (31)
        self.omega_g = float(cfg["omega_g"])
        self.omega_l = float(cfg["omega_l"])
        self.psi_g = float(cfg.get("psi_g", 0.0))
        self.psi_l = float(cfg.get("psi_l", 0.0))
        self.omega_ag = float(cfg["omega_ag"])
        self.omega_al = float(cfg["omega_al"])
        self.drag = cfg.get("drag", "const")
        self.K_I = float(cfg.get("K_I", 0.0))
        self.kappa_I = float(cfg.get("kappa_I", 0.0))
        self.K_W = float(cfg.get("K_W", 0.0))
        self.g_hat = float(cfg.get("g_hat", 0.0))
        self.rho_ref = cfg.get("rho_ref", "liquid")
        self.gamma = float(cfg.get("gamma", 0.0))
        self.n_gamma = int(cfg.get("n_gamma", 1))
        self.alpha_min = float(cfg.get("alpha_min", 1e-6))
        self.alpha_in = (float(cfg.get("alpha_in_max", 0.0)), float(cfg.get("alpha_in_min", 0.0)))
        self.ug_in = (float(cfg.get("ug_in_max", 0.0)), float(cfg.get("ug_in_min", 0.0)))
        self.ul_in = (float(cfg.get("ul_in_max", 0.0)), float(cfg.get("ul_in_min", 0.0)))
        self.n_ramp = float(cfg.get("n_ramp", 0.0))
        self.renormalize = bool(cfg.get("renormalize", True))
        self.sigma_grad = bool(cfg.get("sigma_grad", True))
        # test switch: the slope limiter of reading R13 (always on in the
        # library; off only to show what it prevents)
        self.grad_limiter = bool(cfg.get("grad_limiter", True))


class Oracle:
    """Plain FP64 state of the six schemes on one lattice."""

    def __init__(self, cfg, fields, t0=0):
        """Populations at time t0 rebuilt from the macroscopic fields (the
        initial state when t0 = 0).  Reading R22: a run started (or restarted)
        at t0 takes its lagged S'' and Lambda' at its first step, whatever
        t0 mod n_gamma: the fields carry no lagged values to resume from."""
        p = self.p = Params(cfg)
        lat = self.lat = p.lat
        D = lat.D
        grid = p.shape
        a_g0 = np.asarray(fields["alpha_g"], dtype=np.float64).reshape(grid)
        u_g0 = np.asarray(fields.get("u_g", np.zeros((D,) + grid)), dtype=np.float64).reshape((D,) + grid)
        u_l0 = np.asarray(fields.get("u_l", np.zeros((D,) + grid)), dtype=np.float64).reshape((D,) + grid)
        dp_k0 = np.asarray(fields.get("dp_k", np.zeros(grid)), dtype=np.float64).reshape(grid)
        self.inlet_noise = fields.get("inlet_noise", None)

        # Buoyancy reference density, reading R8: the liquid density (the
        # paper's kinematic pressure, Eqs. (108)-(110)), or the mean mixture
        # density of the initial state, or an explicit value.
        if p.rho_ref == "liquid":
            self.rho_ref = p.rho_l
        elif p.rho_ref == "mixture_mean":
            a_mean = float(np.mean(fields.get("alpha_g_full", a_g0)))
            self.rho_ref = a_mean * p.rho_g + (1.0 - a_mean) * p.rho_l
        else:
            self.rho_ref = float(p.rho_ref)

        self._build_bc_masks()

        # Initial populations (reading R14): local equilibria of the initial
        # macroscopic fields.  eps_g = p_k / c_s^2 (Eq. (111)), eps_l = 1 and
        # phi from Eq. (32).  f_beta is the lattice kinetic scheme's output,
        # so it is built "as streamed" from the equilibria of the initial
        # imposed velocities c_phi, Eqs. (95), (97).
        eps_g0 = 1.0 + dp_k0 / CS2
        eps_l0 = np.ones(grid)
        phi0 = (1.0 / eps_l0) * (1.0 + (eps_g0 - 1.0) / p.R)
        a_l0 = 1.0 - a_g0
        self.f = {
            "g": eq.feq_I(lat, 1.0, eps_g0, u_g0),
            "l": eq.feq_I(lat, phi0, eps_l0, u_l0),
            "ag": eq.feq_S(lat, a_g0, u_g0),
            "al": eq.feq_S(lat, a_l0, u_l0),
        }
        c_g0 = a_l0 * (u_g0 - u_l0)
        c_l0 = a_g0 * (u_l0 - u_g0)
        ones = np.ones(grid)
        bvals0 = {"b_g": ones, "b_l": ones, "c_g": c_g0, "c_l": c_l0}
        self.t = int(t0)
        self.f["bg"] = self._stream("bg", eq.feq_S(lat, ones, c_g0), bvals0, t=self.t - 1)
        self.f["bl"] = self._stream("bl", eq.feq_S(lat, ones, c_l0), bvals0, t=self.t - 1)
        self.lag = None   # taken at the first step (reading R22)

    # ------------------------------------------------------------------ moments
    def moments(self):
        """All moments of the populations at the current time and the
        renormalised volume fractions."""
        lat = self.lat
        v = lat.v.astype(np.float64)
        m = {}
        for ph in ("g", "l"):
            f = self.f[ph]
            m["eps_" + ph] = f.sum(axis=0)                                  # Eq. (40)
            m["u_" + ph] = np.einsum("qc,q...->c...", v, f)                 # Eq. (41)
            m["Pi_" + ph] = np.einsum("qc,qd,q...->cd...", v, v, f)         # text after Eq. (49)
            fa = self.f["a" + ph]
            m["a_" + ph] = fa.sum(axis=0)                                   # Eq. (73)
            m["J_" + ph] = np.einsum("qc,q...->c...", v, fa)                # Eq. (74)
            m["b_" + ph] = self.f["b" + ph].sum(axis=0)                     # Eq. (96)
        if self.p.renormalize:
            # Spalding renormalisation, Eq. (93); reading R2 for B(0) + B(0) = 0.
            Bg, Bl = spalding_B(m["a_g"]), spalding_B(m["a_l"])
            den = Bg + Bl
            safe = np.where(den > 0, den, 1.0)
            m["alpha_g"] = np.where(den > 0, Bg / safe, 0.0)
            m["alpha_l"] = 1.0 - m["alpha_g"]
        else:
            m["alpha_g"] = m["a_g"].copy()
            m["alpha_l"] = m["a_l"].copy()
        # Imposed velocities of the source schemes, Eq. (97) with beta = 1
        # at the start of every step (text before Eq. (105)).
        m["c_g"] = m["alpha_l"] * (m["u_g"] - m["u_l"])
        m["c_l"] = m["alpha_g"] * (m["u_l"] - m["u_g"])
        return m

    # --------------------------------------------------------------------- step
    def step(self, n=1):
        for _ in range(n):
            self._step_once()

    def _step_once(self):
        p, lat = self.p, self.lat
        D = lat.D
        t = self.t
        m = self.moments()
        eps_g, eps_l, u_g, u_l = m["eps_g"], m["eps_l"], m["u_g"], m["u_l"]
        alpha_g, alpha_l = m["alpha_g"], m["alpha_l"]
        I = np.eye(D).reshape((D, D) + (1,) * eps_g.ndim)

        # Liquid equation of state, Eq. (32).
        phi = (1.0 / eps_l) * (1.0 + (eps_g - 1.0) / p.R)

        # Continuity sources from the source schemes, Eq. (107).
        S_g = 1.0 - m["b_g"]
        S_l = 1.0 - m["b_l"]
        # Dashpots: gas Eq. (128); liquid Eq. (131) with the third strategy
        # Gamma_l = phi eps_l - 1.  Reading R11: u^2 -> |u|^2 in several dimensions.
        usq_g = np.sum(u_g * u_g, axis=0)
        usq_l = np.sum(u_l * u_l, axis=0)
        Sp_g = S_g - p.gamma * usq_g * (eps_g - 1.0)
        Sp_l = S_l - p.gamma * usq_l * (phi * eps_l - 1.0)
        # Clift-Grace-Weber volume-fraction factor, Eq. (136).
        Lam = alpha_g * alpha_l * (alpha_g + alpha_l * p.R)
        # Lagged updates, Eqs. (133) and (137); reading R9: refresh when
        # t mod n_gamma == 0, t = 0 included; reading R22: and at the first
        # step of a run.
        if t % p.n_gamma == 0 or self.lag is None:
            self.lag = {"S2_g": Sp_g.copy(), "S2_l": Sp_l.copy(), "Lam": Lam.copy()}
        S2_g, S2_l, Lam_lag = self.lag["S2_g"], self.lag["S2_l"], self.lag["Lam"]

        # Volume-fraction gradients from the f_alpha non-equilibrium flux,
        # Eq. (91) (reading R4: the raw zeroth moment multiplies u), then
        # the symmetrisation of Eq. (94).
        grad_g = (p.omega_ag / CS2) * (m["a_g"] * u_g - m["J_g"])
        grad_l = (p.omega_al / CS2) * (m["a_l"] * u_l - m["J_l"])
        delta = grad_g + grad_l
        grad_g = grad_g - delta / 2.0
        grad_l = grad_l - delta / 2.0

        # Viscous stress from the non-equilibrium second moment, Eq. (70)
        # with Pi^eq of Eq. (50) (phi_g = 1).  Reading R10: the lagged,
        # damped source S'' is the S used here and in G.
        uu_g = np.einsum("c...,d...->cd...", u_g, u_g)
        uu_l = np.einsum("c...,d...->cd...", u_l, u_l)
        Pieq_g = 1.0 * CS2 * eps_g * I + uu_g
        Pieq_l = phi * CS2 * eps_l * I + uu_l
        sig_g = (1.0 / p.omega_g - 0.5) * p.omega_g * (Pieq_g - m["Pi_g"]) - (CS2 * p.psi_g / 2.0) * S2_g * I
        sig_l = (1.0 / p.omega_l - 0.5) * p.omega_l * (Pieq_l - m["Pi_l"]) - (CS2 * p.psi_l / 2.0) * S2_l * I

        # Interphase drag, Eqs. (6) and (135): F_gl / rho_g = K_I |u_l - u_g| (u_l - u_g).
        K_I = p.kappa_I * Lam_lag if p.drag == "cgw" else p.K_I
        du = u_l - u_g
        du_norm = np.sqrt(np.sum(du * du, axis=0))
        F_gl_over_rho_g = K_I * du_norm * du
        # Wall friction of the liquid, Eq. (119) (reading R12: friction, minus sign).
        ul_norm = np.sqrt(usq_l)
        F_l_over_rho_g = p.K_W * ul_norm * (-u_l)
        # Reading R13: the 1/alpha factors use max(alpha, alpha_min).
        ag_f = np.maximum(alpha_g, p.alpha_min)
        al_f = np.maximum(alpha_l, p.alpha_min)
        # Buoyancy, reading R8 (Eqs. (108)-(116) with a general reference density).
        e_up = np.zeros((D,) + (1,) * eps_g.ndim)
        e_up[p.up_axis] = 1.0
        b_g = (self.rho_ref / p.rho_g - 1.0) * p.g_hat
        b_l = (self.rho_ref / p.rho_l - 1.0) * p.g_hat

        # Forces, Eqs. (24) and (26) with F_lg = -F_gl and F_g = 0.
        # Reading R13 (continued): in sigma . grad(alpha) / alpha the
        # gradient is limited to |grad alpha_phi| <= max(alpha_phi, alpha_min)
        # per lattice spacing -- a slope limiter, as the paper proposes for
        # this term where alpha -> 0 (Sec. 2.1): a log-gradient steeper than
        # one per node is not resolved, and at nodes the clamp of Eq. (93)
        # has emptied of a phase the raw flux-based gradient of Eq. (91)
        # would otherwise be divided by alpha_min.
        gnorm = np.sqrt(np.sum(grad_g * grad_g, axis=0))          # |grad alpha_l| = |grad alpha_g|
        lim_g = np.where(gnorm > ag_f, ag_f / np.where(gnorm > 0, gnorm, 1.0), 1.0)
        lim_l = np.where(gnorm > al_f, al_f / np.where(gnorm > 0, gnorm, 1.0), 1.0)
        if not p.grad_limiter:
            lim_g = lim_l = 1.0
        sgrad_g = np.einsum("cd...,d...->c...", sig_g, grad_g * lim_g) / ag_f
        sgrad_l = np.einsum("cd...,d...->c...", sig_l, grad_l * lim_l) / al_f
        if not p.sigma_grad:
            sgrad_g = np.zeros_like(sgrad_g)
            sgrad_l = np.zeros_like(sgrad_l)
        G_g = S2_g * u_g + sgrad_g + b_g * e_up + F_gl_over_rho_g / ag_f
        G_l = S2_l * u_l + sgrad_l + b_l * e_up + (-F_gl_over_rho_g + F_l_over_rho_g) / (al_f * p.R)

        # Collision and forcing of the momentum schemes, Eqs. (34)-(37), (42).
        fs = {}
        fs["g"] = self.f["g"] + p.omega_g * (eq.feq_I(lat, 1.0, eps_g, u_g) - self.f["g"]) \
            + eq.feq_L(lat, p.psi_g, S2_g, G_g)
        fs["l"] = self.f["l"] + p.omega_l * (eq.feq_I(lat, phi, eps_l, u_l) - self.f["l"]) \
            + eq.feq_L(lat, p.psi_l, S2_l, G_l)
        # Volume-fraction schemes, Eqs. (71)-(72), with the renormalised
        # alpha (reading R3).
        fs["ag"] = self.f["ag"] + p.omega_ag * (eq.feq_S(lat, alpha_g, u_g) - self.f["ag"])
        fs["al"] = self.f["al"] + p.omega_al * (eq.feq_S(lat, alpha_l, u_l) - self.f["al"])
        # Source schemes: lattice kinetic scheme, Eq. (95), beta = 1.
        ones = np.ones_like(eps_g)
        fs["bg"] = eq.feq_S(lat, ones, m["c_g"])
        fs["bl"] = eq.feq_S(lat, ones, m["c_l"])

        # Intermediate quantities of this step, kept for the budget tests.
        self.last = dict(m=m, S_g=S_g, S_l=S_l, S2_g=S2_g, S2_l=S2_l, G_g=G_g, G_l=G_l,
                         grad_g=grad_g, grad_l=grad_l, sig_g=sig_g, sig_l=sig_l, phi=phi,
                         drag_g=F_gl_over_rho_g / ag_f, drag_l=-F_gl_over_rho_g / (al_f * p.R))
        for s in SCHEMES:
            self.f[s] = self._stream(s, fs[s], m, t=t)
        self.t = t + 1

    # ----------------------------------------------------------------- boundary
    def _build_bc_masks(self):
        """For every direction q, the nodes whose upstream neighbour x - v_q
        lies outside the domain, grouped by the rule that fills them.

        Reading R15: a population arriving through a wall face (also the
        diagonal ones at a corner) takes the wall rule; one arriving only
        through an inlet or outlet face takes that face's rule."""
        p, lat = self.p, self.lat
        D = lat.D
        grid = p.shape
        idx = np.indices(grid)                              # idx[a] along array axis a
        self.masks = []
        for q in range(lat.Q):
            faces = []
            for c in range(D):
                ax = D - 1 - c
                n = grid[ax]
                name = "xyz"[c]
                if lat.v[q, c] == 1 and p.bc[name + "-"] != "periodic":
                    faces.append((name + "-", idx[ax] == 0))
                if lat.v[q, c] == -1 and p.bc[name + "+"] != "periodic":
                    faces.append((name + "+", idx[ax] == n - 1))
            wall = np.zeros(grid, dtype=bool)
            opn = np.zeros(grid, dtype=bool)
            for face, on in faces:
                if p.bc[face] == "wall":
                    wall |= on
                elif p.bc[face] == "open":
                    opn |= on
            opn &= ~wall
            per_face = []
            taken = wall | opn
            for face, on in faces:
                if p.bc[face] in ("inlet", "outlet"):
                    msk = on & ~taken
                    taken = taken | msk
                    per_face.append((face, msk))
            self.masks.append((wall, opn, per_face))

    def _face_values(self, y, face, mode, idx):
        """STEP #1 of Sec. 3.5, Eqs. (160)-(161): the nodal field y extrapolated
        to a boundary face, half-way (hw) or full-way (fw), for the nodes idx
        (a tuple of grid index arrays) lying on that face; extrapolation runs
        along the face normal from the edge node and its inward neighbour."""
        D = self.lat.D
        c = FACE_AXES[face[0]]
        ax = D - 1 - c
        n = self.p.shape[ax]
        e, nxt = (0, 1) if face[1] == "-" else (n - 1, n - 2)
        ie = tuple(np.full_like(ix, e) if a == ax else ix for a, ix in enumerate(idx))
        iN = tuple(np.full_like(ix, nxt) if a == ax else ix for a, ix in enumerate(idx))
        lead = (slice(None),) * (y.ndim - D)
        ye, yn = y[lead + ie], y[lead + iN]
        return 1.5 * ye - 0.5 * yn if mode == "hw" else 2.0 * ye - yn

    def _inlet_dir(self, face, m):
        """Unit normal of an inlet face pointing into the domain, for m nodes."""
        D = self.lat.D
        nvec = np.zeros((D, m))
        nvec[FACE_AXES[face[0]]] = 1.0 if face[1] == "-" else -1.0
        return nvec

    def _inlet_alpha(self, face, t, idx):
        """Inlet gas fraction at time t: the ramp of Eq. (153) times the
        per-node factor of the inlet face (reading R17)."""
        p = self.p
        a_in = _ramp(t, p.alpha_in[0], p.alpha_in[1], p.n_ramp)
        if self.inlet_noise is None:
            return np.full(idx[0].shape, a_in)
        ax = self.lat.D - 1 - FACE_AXES[face[0]]
        noise = np.asarray(self.inlet_noise, dtype=np.float64)
        return a_in * noise[tuple(ix for a, ix in enumerate(idx) if a != ax)]

    def _stream(self, s, fstar, m, t):
        """Streaming (left-hand sides of Eqs. (34), (35), (71), (95)) plus
        STEP #2 of Sec. 3.5 for the populations entering through a face."""
        p, lat = self.p, self.lat
        D = lat.D
        out = np.empty_like(fstar)
        axes = tuple(D - 1 - c for c in range(D))
        for q in range(lat.Q):
            out[q] = np.roll(fstar[q], shift=tuple(int(lat.v[q, c]) for c in range(D)), axis=axes)
        if all(b == "periodic" for b in p.bc.values()):
            return out
        phase = s[-1]
        for q in range(lat.Q):
            wall, opn, per_face = self.masks[q]
            qs = lat.opp[q]                                  # q* leaves the domain, q = BB(q*)
            if wall.any():
                if s in ("bg", "bl"):
                    # EQ(S) with beta = 1, c = 0 at a wall (reading R15).
                    k = int(wall.sum())
                    out[q][wall] = eq.feq_S(lat, np.ones(k), np.zeros((D, k)))[q]
                else:
                    # Half-way bounce-back with zero wall velocity (reading R15).
                    out[q][wall] = fstar[qs][wall]
            if opn.any():
                out[q][opn] = fstar[q][opn]
            for face, msk in per_face:
                idx = np.nonzero(msk)
                k = idx[0].size
                if k == 0:
                    continue
                kind = p.bc[face]
                fo = fstar[qs][idx]                          # f*(x_E, t, q*)
                if s in ("bg", "bl"):
                    # EQ(S), beta and c extrapolated full-way (Tables 1-2).
                    # Reading R16: the beta extrapolated is the one the
                    # equilibria of the source schemes carry, beta = 1 at the
                    # start of every step at every node (text before
                    # Eq. (105)), so the missing node emits f^eq(1, c_B).
                    # (Extrapolating the post-streaming moment 1 - S instead
                    # feeds S back into itself with gain 2 sum_q w_q at the
                    # face: S grows about 1.5x per node towards an outlet and,
                    # with the lag of Eq. (133), the tube of TEST #3 diverges
                    # at t ~ 3.7e4.)
                    bB = np.ones(k)
                    cB = self._face_values(m["c_" + phase], face, "fw", idx)
                    val = eq.feq_S(lat, bB, cB)[q]
                elif kind == "inlet":
                    nvec = self._inlet_dir(face, k)
                    if s in ("g", "l"):
                        # BB(I), Eq. (163): eps extrapolated half-way, u imposed.
                        uin = (_ramp(t, *p.ug_in, p.n_ramp) if phase == "g" else _ramp(t, *p.ul_in, p.n_ramp))
                        uB = uin * nvec
                        epsB = self._face_values(m["eps_" + phase], face, "hw", idx)
                        if phase == "g":
                            phiB = np.ones(k)
                        else:
                            eg = self._face_values(m["eps_g"], face, "hw", idx)
                            phiB = (1.0 / epsB) * (1.0 + (eg - 1.0) / p.R)
                        delta = eq.feq_I(lat, phiB, epsB, -uB)[qs] - eq.feq_I(lat, phiB, epsB, uB)[qs]
                        val = fo + delta
                    else:
                        # EQ(S) with the imposed alpha and u.
                        a_in = self._inlet_alpha(face, t, idx)
                        if phase == "g":
                            aB, uin = a_in, _ramp(t, *p.ug_in, p.n_ramp)
                        else:
                            aB, uin = 1.0 - a_in, _ramp(t, *p.ul_in, p.n_ramp)
                        val = eq.feq_S(lat, aB, uin * nvec)[q]
                else:  # outlet
                    uB = self._face_values(m["u_" + phase], face, "hw", idx)
                    if s in ("g", "l"):
                        # ABB(I), Eq. (164): eps = 1 (hence phi = 1), u extrapolated half-way.
                        one = np.ones(k)
                        delta = eq.feq_I(lat, one, one, -uB)[qs] + eq.feq_I(lat, one, one, uB)[qs]
                    else:
                        # ABB(S): alpha and u extrapolated half-way.
                        aB = self._face_values(m["alpha_" + phase], face, "hw", idx)
                        delta = eq.feq_S(lat, aB, -uB)[qs] + eq.feq_S(lat, aB, uB)[qs]
                    val = -fo + delta
                out[q][idx] = val
        return out

    # ----------------------------------------------------------------- read-out
    def read(self):
        """Macroscopic fields at the current time: renormalised volume
        fractions, phase velocities and the kinematic pressure p_k = c_s^2 eps_g
        (Eq. (111)), also as its deviation from c_s^2."""
        m = self.moments()
        return {
            "alpha_g": m["alpha_g"], "alpha_l": m["alpha_l"],
            "u_g": m["u_g"], "u_l": m["u_l"],
            "p_k": CS2 * m["eps_g"], "dp_k": CS2 * (m["eps_g"] - 1.0),
        }

    def diag(self):
        """Domain sums at the current time (conservation budgets)."""
        m = self.moments()
        p = self.p
        mom = p.rho_g * m["alpha_g"] * m["u_g"] + p.rho_l * m["alpha_l"] * m["u_l"]
        allf = np.concatenate([self.f[s].ravel() for s in SCHEMES])
        sum_axes = tuple(range(1, 1 + self.lat.D))
        return {
            "a_g": float(m["a_g"].sum()), "a_l": float(m["a_l"].sum()),
            "alpha_g": float(m["alpha_g"].sum()), "alpha_l": float(m["alpha_l"].sum()),
            "eps_g": float(m["eps_g"].sum()), "eps_l": float(m["eps_l"].sum()),
            "u_g": m["u_g"].sum(axis=sum_axes), "u_l": m["u_l"].sum(axis=sum_axes),
            "momentum": mom.sum(axis=sum_axes),
            "renorm_defect": float((m["alpha_g"] - m["a_g"]).sum()),
            "nonfinite": int(np.count_nonzero(~np.isfinite(allf))),
        }
