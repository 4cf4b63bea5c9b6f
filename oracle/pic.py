"""FP64 oracle of the 1D3V PIC/MCC cycle (Sec. IV and IV.A, Fig. 4).

One time step l -> l+1, in the order of the paper's simulation cycle:
  1. charge assignment: linear (cloud-in-cell) weighting onto the two nearest
     nodes ('Charge Assignment'), accumulated as integers in units of 2^-32 of a
     super-particle so the result does not depend on summation order;
  2. field solve: second-order finite-difference Poisson equation with the
     driven electrode potential V(t_l) at x = 0 and ground at x = L, then
     E_m = -(Phi_{m+1} - Phi_{m-1}) / (2 dx) ('EM Field Solver');
  3. field interpolation: linear weighting back to the particle ('Field
     Interpolation');
  4. push: leapfrog Eqs. (3)-(4) with a = (q/m) E ('Particle Pushing');
  5. walls: particles leaving [0, L) are absorbed; ion impact energy and angle
     are recorded per electrode ('Wall Interaction');
  6. Monte Carlo collisions with the null-collision method, Eq. (6) and the
     process selection that follows it ('Particle Collisions').

State: positions are kept in cell units xt = x / dx (node m sits at xt = m),
velocities in m/s (3 components: '1D3V').  Super-particle weight w = n0 L / N_p
(particles per m^2) is shared by electrons and ions (Sec. IV, weight w = q/Q).

Readings taken where the paper is silent (each also listed in the design notes):
  * V(t) = V0 cos(omega t + phi) on the left electrode, right electrode grounded,
    no blocking capacitor (the workloads' single sinusoid);
  * boundary-node volumes are dx/2; boundary fields use Gauss's law over that
    half cell, E_0 = (Phi_0 - Phi_1)/dx - rho_0 dx/(2 eps0) and
    E_N = (Phi_{N-1} - Phi_N)/dx + rho_N dx/(2 eps0);
  * loaded velocities are v^(-1/2) (no initial half-step pull-back);
  * absorbed iff xt < 0 or xt >= N (half-open domain);
  * nu_max of Eq. (6) is the maximum of n sigma_sum(eps) g over eps in
    (0, E_cap] (the literal maximum over all energies is unbounded for a
    constant elastic cross section); faster particles still use it and are
    counted as overflows;
  * electrons see the gas at rest, ions draw a Maxwellian partner (Sec. IV);
  * the per-step collision check R <= P_c,tot is drawn as a geometric waiting
    time (same law, see ``skip``); by default the wait is the plain geometric
    one.  ``Discharge(wait_cap=WAIT_CAP)`` cuts waits longer than WAIT_CAP
    steps and redraws them at the cut (the same law, since the geometric law
    has no memory): the GPU stores a particle's next examination step in 15
    bits and works that way, and single-step parity from a GPU state needs the
    oracle to take the same schedule;
  * selection intervals are half-open [S_{j-1}, S_j), process order
    elastic, excitation, ionisation;
  * ionisation: both electrons share eps - E_ion equally with independent
    isotropic directions; the new ion is Maxwellian at the gas temperature;
  * electron elastic and excitation scattering are isotropic in the centre of
    mass frame (VHS-like, Eq. (10) with chi = 2 arccos(b / b_max));
  * phase-resolved averages bin step l by its RF phase, floor((l mod N_t)
    n_phase / N_t); the flux profiles of Fig. 8 are sampled from the state a
    step starts from (x^(l) with v_x^(l-1/2)), the same positions as that
    step's charge, so that Gamma / n is a mean velocity of the same particles.
"""
import math
import numpy as np

from . import constants as C
from . import philox as R
from .xsec import electron_sigmas

TWO32 = 2 ** 32
NEVER = 2 ** 32 - 1          # "no further candidate" marker of the skip schedule
WAIT_CAP = 32767             # longest wait of the cut schedule (Discharge(wait_cap=WAIT_CAP))

# flags (test modes grounded in the paper: collisionless / field-free runs)
NO_SELF_FIELD = 1
NO_COLLISIONS = 2

# electron process ids in selection order; ion charge exchange
P_EL, P_EXC, P_ION, P_NULL = 0, 1, 2, 3
P_CX = 0

# status codes (same meaning as the C interface)
OK, ECAPACITY, ENUMERIC = 0, -4, -5

N_ANGLE_BINS = 360            # 0.25 degree bins over [0, 90) degrees
ANGLE_BIN_DEG = 0.25
# joint energy-angle histogram of the ion impacts (Fig. 7): 4 eV by 1 degree
IEAD_E_GROUP = 4              # 1 eV bins per energy bin
IEAD_A_GROUP = 4              # 0.25 degree bins per angle bin
IEAD_A_BINS = N_ANGLE_BINS // IEAD_A_GROUP

WARN_DEBYE, WARN_PLASMA_FREQ, WARN_PPC = 1, 2, 4


def derived(p):
    """Quantities derived from the case parameters (host-side set-up)."""
    d = {}
    N = int(p["n_cells"])
    L = float(p["gap_m"])
    d["N"] = N
    d["dx"] = L / N
    d["dt"] = 1.0 / (p["freq_hz"] * p["steps_per_cycle"])
    d["n_gas"] = C.gas_density(p["p_pa"], p["t_gas_k"])
    d["w"] = p["n0_m3"] * L / p["np_e"]
    d["m"] = (C.M_E, C.M_AR)
    d["q"] = (-C.E_CHARGE, C.E_CHARGE)
    d["mr"] = (C.M_E * C.M_AR / (C.M_E + C.M_AR), 0.5 * C.M_AR)
    d["nu_max"] = (nu_max_electron(p, d), nu_max_ion(p, d))
    if p.get("flags", 0) & NO_COLLISIONS or p["p_pa"] == 0:
        d["p_tot"] = (0.0, 0.0)
    else:
        d["p_tot"] = tuple(-math.expm1(-nu * d["dt"]) for nu in d["nu_max"])
    d["n_ebins"] = int(math.ceil(p["ecap_i_ev"]))     # 1 eV ion energy bins
    # Sec. IV.A 'Limitations and Constraints': dx << lambda_D, dt << 1/omega_p,
    # N_C >= 20 super-particles per cell; violations are warnings, not errors
    lam_d = math.sqrt(C.EPS0 * p["te_ev"] / (p["n0_m3"] * C.E_CHARGE))
    omega_p = math.sqrt(p["n0_m3"] * C.E_CHARGE ** 2 / (C.EPS0 * C.M_E))
    warn = 0
    if d["dx"] > lam_d:
        warn |= WARN_DEBYE
    if omega_p * d["dt"] > 0.2:
        warn |= WARN_PLASMA_FREQ
    if p["np_e"] / N < 20:
        warn |= WARN_PPC
    d["warnings"] = warn
    return d


def nu_sum_electron(eps_ev, p, n_gas):
    """n_bg sigma_sum(eps) sqrt(2 eps / m_r) for electrons (Eq. (6) before the max)."""
    mr = C.M_E * C.M_AR / (C.M_E + C.M_AR)
    xs = p
    s_el, s_exc, s_ion = electron_sigmas(eps_ev, xs)
    g = np.sqrt(2.0 * np.asarray(eps_ev) * C.E_CHARGE / mr)
    return n_gas * (s_el + s_exc + s_ion) * g


def nu_max_electron(p, d):
    """Eq. (6): maximum over eps in (0, E_cap,e] on a 4096-point uniform grid."""
    eps = p["ecap_e_ev"] * np.arange(1, 4097) / 4096.0
    return float(np.max(nu_sum_electron(eps, p, d["n_gas"])))


def nu_max_ion(p, d):
    """Eq. (6) for Ar+ charge exchange with a constant cross section: the largest
    relative speed is the capped ion speed plus ten thermal partner widths."""
    g_cap = math.sqrt(2.0 * p["ecap_i_ev"] * C.E_CHARGE / C.M_AR) \
        + 10.0 * math.sqrt(C.K_B * p["t_gas_k"] / C.M_AR)
    return d["n_gas"] * p["sigma_cx"] * g_cap


def skip(U, step, p_tot, wait_cap=None):
    """Next examination step of the null-collision schedule.

    The paper tests R_f <= P_c,tot once per step (Sec. IV and Eq. (6)).  Those
    tests are independent Bernoulli(P_c,tot) trials, so the number of steps to
    the next success is geometric: G = ceil(ln U / ln(1 - P_c,tot)) >= 1.  With
    a wait_cap, a wait longer than wait_cap steps is cut at wait_cap: the
    particle is then examined without a collision test and draws a fresh wait
    ('redraw').  The geometric law has no memory -- P(G > a + b | G > a) =
    P(G > b) -- so the steps of the real tests keep the law of independent
    per-step trials either way.
    Returns (next step, redraw flag, near-tie flag); the last marks draws whose
    ratio lies within 1e-9 (relative) of an integer, the only ones where FP64
    libraries may round to a different G.  Without collisions: NEVER."""
    step = np.asarray(step, dtype=np.int64)
    if p_tot <= 0.0:
        return (np.full(U.shape, NEVER, dtype=np.int64), np.zeros(U.shape, bool), np.zeros(U.shape, bool))
    ratio = np.log(U) / math.log1p(-p_tot)
    G = np.maximum(np.ceil(ratio), 1.0)
    tie = np.abs(ratio - np.rint(ratio)) < 1e-9 * np.maximum(ratio, 1.0)
    if wait_cap is None:
        redraw = np.zeros(G.shape, dtype=bool)
        return step + G.astype(np.int64), redraw, tie
    redraw = G > wait_cap
    nxt = step + np.where(redraw, wait_cap, G).astype(np.int64)
    return nxt, redraw, tie


def isotropic_direction(Ua, Ub):
    """Unit vector from the impact-parameter sampling of Eq. (10) under the VHS
    scattering law: b/b_max = sqrt(R), chi = 2 arccos(b/b_max), psi = 2 pi R."""
    b_over_bmax = np.sqrt(Ua)
    chi = 2.0 * np.arccos(b_over_bmax)
    psi = 2.0 * np.pi * Ub
    return np.stack([np.cos(chi), np.sin(chi) * np.cos(psi), np.sin(chi) * np.sin(psi)], axis=-1)


def deposit(xt, N):
    """Linear (cloud-in-cell) charge assignment in integer units of 2^-32 particle.

    Node j = floor(xt) receives 2^32 - W and node j+1 receives W with
    W = rint((xt - j) 2^32), so every super-particle deposits exactly 2^32."""
    xt = np.asarray(xt, dtype=np.float64)
    j = np.floor(xt).astype(np.int64)
    W = np.rint((xt - j) * TWO32).astype(np.int64)
    Q = np.zeros(N + 1, dtype=np.int64)
    np.add.at(Q, j, TWO32 - W)
    np.add.at(Q, j + 1, W)
    return Q


def flux_weights(xt, vx, N):
    """Particle flux sample: sum over particles of S_m(xt) v_x at every node m,
    with S_m the same linear weighting as the charge (node floor(xt) gets 1 - f,
    the next node f, f = xt - floor(xt)).  Times w / vol_m this is the flux
    density n u of the sample (Fig. 8's flux profiles)."""
    xt = np.asarray(xt, dtype=np.float64)
    vx = np.asarray(vx, dtype=np.float64)
    j = np.floor(xt).astype(np.int64)
    f = xt - j
    F = np.zeros(N + 1)
    np.add.at(F, j, (1.0 - f) * vx)
    np.add.at(F, j + 1, f * vx)
    return F


def phase_bin(l, steps_per_cycle, n_phase):
    """RF phase bin of step l: the phase (l mod N_t) / N_t cut into n_phase equal
    bins (phase-resolved averaging, Sec. IV)."""
    return ((l % steps_per_cycle) * n_phase) // steps_per_cycle


def charge_density(Qe, Qi, w, dx, N):
    """rho_m = e w (Q_i - Q_e)_m / (2^32 dx_m); boundary nodes own half a cell."""
    vol = np.full(N + 1, dx)
    vol[0] = vol[N] = 0.5 * dx
    return C.E_CHARGE * w * (Qi - Qe).astype(np.float64) / (TWO32 * vol)


def solve_potential(rho, V, dx):
    """(Phi_{m+1} - 2 Phi_m + Phi_{m-1}) / dx^2 = -rho_m / eps0 for m = 1..N-1 with
    Phi_0 = V and Phi_N = 0, solved as a banded (tridiagonal) system."""
    from scipy.linalg import solve_banded
    N = rho.size - 1
    Phi = np.zeros(N + 1)
    Phi[0] = V
    if N == 1:
        return Phi
    n = N - 1
    ab = np.zeros((3, n))
    ab[0, 1:] = 1.0
    ab[1, :] = -2.0
    ab[2, :-1] = 1.0
    b = -rho[1:N] * dx * dx / C.EPS0
    b[0] -= V
    Phi[1:N] = solve_banded((1, 1), ab, b)
    return Phi


def solve_potential_circuit(rho, dx, cb, sigma_rhs):
    """The driven electrode behind a blocking capacitor (Sec. III: the source
    reaches the left electrode through C_B; Sec. IV.A 'EM Field Solver and
    External Lumped Circuits': the electrode's surface charge is the interface to
    the circuit).  Unknowns Phi_0..Phi_{N-1} (Phi_N = 0): Poisson's equation for
    m = 1..N-1 and, at m = 0, the surface charge from Gauss's law over the half
    cell, eps0 (Phi_0 - Phi_1) / dx - rho_0 dx / 2, equal to what the circuit
    has delivered: sigma_rhs - cb Phi_0 with sigma_rhs = sigma_init + cb V(t_l)
    + q_abs (the capacitor starts uncharged at the load; q_abs is the net charge
    the electrode has absorbed from particles, per area).  cb in F/m^2.  One
    banded system."""
    from scipy.linalg import solve_banded
    N = rho.size - 1
    a = C.EPS0 / dx
    Phi = np.zeros(N + 1)
    if N == 1:
        Phi[0] = (sigma_rhs + rho[0] * dx / 2) / (a + cb)
        return Phi
    ab = np.zeros((3, N))
    ab[0, 1:] = 1.0
    ab[0, 1] = -a
    ab[1, :] = -2.0
    ab[1, 0] = a + cb
    ab[2, :-1] = 1.0
    b = -rho[:N] * dx * dx / C.EPS0
    b[0] = sigma_rhs + rho[0] * dx / 2
    Phi[:N] = solve_banded((1, 1), ab, b)
    return Phi


def electric_field(Phi, rho, dx):
    """E_m = -(Phi_{m+1} - Phi_{m-1}) / (2 dx) inside; Gauss's law over the half
    cell at the two electrodes."""
    N = Phi.size - 1
    E = np.empty(N + 1)
    E[1:N] = -(Phi[2:] - Phi[:-2]) / (2.0 * dx)
    E[0] = (Phi[0] - Phi[1]) / dx - rho[0] * dx / (2.0 * C.EPS0)
    E[N] = (Phi[N - 1] - Phi[N]) / dx + rho[N] * dx / (2.0 * C.EPS0)
    return E


def gather(E, xt):
    """Linear interpolation of the nodal field to the particle (same weights as
    the charge assignment)."""
    j = np.floor(xt).astype(np.int64)
    f = xt - j
    return (1.0 - f) * E[j] + f * E[j + 1]


def voltage(p, step):
    """Source voltage V(t_l) = V0 cos(wt + phi) + V2 cos(2wt + phi2), wt = 2 pi
    (l mod N_t) / N_t: a fundamental and its harmonic, the electrical-asymmetry
    drive of Sec. III (V2 = V0, phi2 = 0 there; V2 = 0 a single sinusoid)."""
    Nt = int(p["steps_per_cycle"])
    wt = 2.0 * math.pi * (int(step) % Nt) / Nt
    return (p["v0_volt"] * math.cos(wt + p["phase_rad"])
            + p.get("v2_volt", 0.0) * math.cos(2.0 * wt + p.get("phase2_rad", 0.0)))


class Species:
    def __init__(self, n):
        self.xt = np.zeros(n)
        self.v = np.zeros((n, 3))
        self.id = np.zeros(n, dtype=np.uint64)
        self.next = np.zeros(n, dtype=np.int64)
        self.redraw = np.zeros(n, dtype=bool)     # the next examination only redraws the wait

    def __len__(self):
        return self.xt.size

    def take(self, keep):
        self.xt, self.v, self.id = self.xt[keep], self.v[keep], self.id[keep]
        self.next, self.redraw = self.next[keep], self.redraw[keep]

    def append(self, xt, v, ids, nxt, redraw):
        self.xt = np.concatenate([self.xt, xt])
        self.v = np.concatenate([self.v, v])
        self.id = np.concatenate([self.id, ids])
        self.next = np.concatenate([self.next, nxt])
        self.redraw = np.concatenate([self.redraw, redraw])


class Discharge:
    """One discharge case.  ``p`` is the case parameter dict (same fields as the
    C interface's case parameters).  wait_cap: None for the plain geometric
    waits of the per-step collision check, or the cut of ``skip``."""

    def __init__(self, p, load=True, wait_cap=None):
        self.p = dict(p)
        self.wait_cap = wait_cap
        self.d = derived(self.p)
        self.step_index = 0
        self.status = OK
        self.sp = [Species(0), Species(0)]
        # blocking-capacitor circuit: the driven electrode's surface charge at the
        # first field solve, and ions minus electrons it has absorbed since
        self.sigma_init = None
        self.n_abs_net = 0
        self.reset_diagnostics()
        if load:
            self.load()

    # ---------------------------------------------------------------- loading
    def load(self):
        """Initial loading (Sec. IV): uniform positions, Maxwellian velocities by
        Box-Muller, and the first candidate step of each particle."""
        p, d = self.p, self.d
        for s, (n, T_ev, m) in enumerate([(p["np_e"], p["te_ev"], C.M_E),
                                          (p["np_i"], p["ti_ev"], C.M_AR)]):
            ids = np.arange(n, dtype=np.uint64)
            U = R.draw(ids, 0, R.tag(s, R.INIT), p["seed"], p["case_id"])
            sp = Species(0)
            sp.xt = d["N"] * U[:, 0]
            sp.v = R.maxwell_velocity(U[:, 1:5], math.sqrt(T_ev * C.E_CHARGE / m))
            sp.id = ids
            Us = R.draw(ids, np.uint64(2 ** 64 - 1), R.tag(s, R.SKIP), p["seed"], p["case_id"])
            sp.next, sp.redraw, _ = skip(Us[:, 0], -1, d["p_tot"][s], self.wait_cap)
            self.sp[s] = sp

    # ------------------------------------------------------------ diagnostics
    def reset_diagnostics(self):
        N = self.d["N"]
        nb = self.d["n_ebins"]
        nph = int(self.p.get("n_phase", 0))
        nf = max(nph, 1) if self.p.get("flux_profiles", 0) else 0
        self.acc = {
            # phase-resolved sums (bin of each step) and flux samples
            "sumQ_phase": np.zeros((nph, 2, N + 1), dtype=np.int64),
            "sumPhi_phase": np.zeros((nph, N + 1)),
            "n_phase": np.zeros(nph, dtype=np.int64),
            "sumF": np.zeros((nf, 2, N + 1)),
            "n_flux": np.zeros(nf, dtype=np.int64),
            "n_steps": 0,
            "sumQ": np.zeros((2, N + 1), dtype=np.int64),
            "sumPhi": np.zeros(N + 1),
            "absorbed": np.zeros((2, 2), dtype=np.int64),        # [species][electrode]
            "iedf": np.zeros((2, nb), dtype=np.int64),           # Ar+ energy, 1 eV bins
            "iadf": np.zeros((2, N_ANGLE_BINS), dtype=np.int64),  # Ar+ angle, 0.25 deg
            "iead": np.zeros((2, -(-nb // IEAD_E_GROUP), IEAD_A_BINS), dtype=np.int64),  # 4 eV x 1 deg
            "ion_energy_sum": np.zeros(2),
            "collisions": np.zeros(5, dtype=np.int64),           # el, exc, ion, (null), cx
            "candidates": np.zeros(2, dtype=np.int64),
            "overflow": np.zeros(2, dtype=np.int64),
            "births": 0,
            "redraws": np.zeros(2, dtype=np.int64),               # examinations at a cut wait
            "particle_steps": 0,
        }

    def sample_diagnostics(self):
        """Time averages over the steps since the last reset (Sec. IV: averaging
        over an adequate period once steady state is reached)."""
        p, d, a = self.p, self.d, self.acc
        N, dx, w = d["N"], d["dx"], d["w"]
        n = max(a["n_steps"], 1)
        vol = np.full(N + 1, dx)
        vol[0] = vol[N] = 0.5 * dx
        out = {
            "step": self.step_index, "status": self.status, "warnings": d["warnings"],
            "n_e": len(self.sp[0]), "n_i": len(self.sp[1]), "avg_steps": a["n_steps"],
            "ne": w * a["sumQ"][0] / (TWO32 * vol * n),
            "ni": w * a["sumQ"][1] / (TWO32 * vol * n),
            "phi": a["sumPhi"] / n,
            "iedf": a["iedf"].copy(), "iadf": a["iadf"].copy(), "iead": a["iead"].copy(),
            "absorbed": a["absorbed"].copy(),
            "flux": a["absorbed"] * w / (n * d["dt"]),
            "mean_ion_energy": a["ion_energy_sum"] / np.maximum(a["absorbed"][1], 1),
            "collisions": a["collisions"].copy(), "candidates": a["candidates"].copy(),
            "overflow": a["overflow"].copy(), "births": a["births"],
            "particle_steps": a["particle_steps"], "redraws": a["redraws"].copy(),
        }
        out.update(self._flux_profiles(range(a["sumF"].shape[0]), out["ne"], out["ni"]))
        return out

    def _flux_profiles(self, bins, ne, ni):
        """Flux profiles Gamma_s = w sum(S_m v_x) / (vol_m n_samples) over the
        given bins, and the mean velocities Gamma_s / n_s (0 where n_s = 0)."""
        d, a = self.d, self.acc
        N, dx, w = d["N"], d["dx"], d["w"]
        vol = np.full(N + 1, dx)
        vol[0] = vol[N] = 0.5 * dx
        out = {}
        bins = list(bins)
        n_f = int(sum(a["n_flux"][b] for b in bins))
        for s, key, dens in ((0, "e", ne), (1, "i", ni)):
            F = sum((a["sumF"][b][s] for b in bins), np.zeros(N + 1))
            g = w * F / (vol * n_f) if n_f > 0 else np.zeros(N + 1)
            out["gamma_" + key] = g
            out["u_" + key] = np.divide(g, dens, out=np.zeros(N + 1), where=dens > 0)
        return out

    def sample_phase(self, b):
        """Averages over the window's steps in RF phase bin b (Sec. IV:
        phase-resolved averaging): densities, potential, flux profiles and mean
        velocities."""
        d, a = self.d, self.acc
        N, dx, w = d["N"], d["dx"], d["w"]
        n = max(int(a["n_phase"][b]), 1)
        vol = np.full(N + 1, dx)
        vol[0] = vol[N] = 0.5 * dx
        out = {"n_steps": int(a["n_phase"][b]),
               "n_flux_samples": int(a["n_flux"][b]) if a["n_flux"].size else 0,
               "ne": w * a["sumQ_phase"][b][0] / (TWO32 * vol * n),
               "ni": w * a["sumQ_phase"][b][1] / (TWO32 * vol * n),
               "phi": a["sumPhi_phase"][b] / n}
        out.update(self._flux_profiles([b] if a["sumF"].shape[0] else [], out["ne"], out["ni"]))
        return out

    # ------------------------------------------------------------------ field
    def field(self, step):
        p, d = self.p, self.d
        N, dx = d["N"], d["dx"]
        Qe = deposit(self.sp[0].xt, N)
        Qi = deposit(self.sp[1].xt, N)
        if p.get("flags", 0) & NO_SELF_FIELD:
            rho = np.zeros(N + 1)
        else:
            rho = charge_density(Qe, Qi, d["w"], dx, N)
        V = voltage(p, step)
        cb = p.get("cb_f_m2", 0.0)
        if cb > 0.0 and self.sigma_init is not None:
            q_abs = C.E_CHARGE * d["w"] * self.n_abs_net
            Phi = solve_potential_circuit(rho, dx, cb, self.sigma_init + cb * V + q_abs)
        else:
            Phi = solve_potential(rho, V, dx)        # ideal source (or the uncharged start)
        E = electric_field(Phi, rho, dx)
        if cb > 0.0 and self.sigma_init is None:
            self.sigma_init = C.EPS0 * E[0]
        return Qe, Qi, rho, V, Phi, E

    # ------------------------------------------------------------------- step
    def step(self, record=False):
        """Advance one time step; returns a record of intermediate results."""
        p, d, a = self.p, self.d, self.acc
        l = self.step_index
        N, dx, dt = d["N"], d["dx"], d["dt"]
        rec = {"step": l}
        nph = int(p.get("n_phase", 0))
        b = phase_bin(l, p["steps_per_cycle"], nph) if nph > 0 else -1

        # flux sample of the state the step starts from: x^(l), v_x^(l-1/2)
        if p.get("flux_profiles", 0):
            bf = max(b, 0)
            for s in (0, 1):
                a["sumF"][bf][s] += flux_weights(self.sp[s].xt, self.sp[s].v[:, 0], N)
            a["n_flux"][bf] += 1

        # 1-2. charge assignment and field solve at t_l
        Qe, Qi, rho, V, Phi, E = self.field(l)
        if record:
            rec.update(Qe=Qe, Qi=Qi, rho=rho, V=V, Phi=Phi, E=E)
        a["sumQ"][0] += Qe
        a["sumQ"][1] += Qi
        a["sumPhi"] += Phi
        a["n_steps"] += 1
        if b >= 0:
            a["sumQ_phase"][b][0] += Qe
            a["sumQ_phase"][b][1] += Qi
            a["sumPhi_phase"][b] += Phi
            a["n_phase"][b] += 1

        births = []
        for s in (0, 1):
            sp = self.sp[s]
            a["particle_steps"] += len(sp)
            if not np.all(np.isfinite(sp.xt)) or not np.all(np.isfinite(sp.v)):
                self.status = ENUMERIC
            # 3-4. gather and leapfrog push, Eqs. (3)-(4)
            Ep = gather(E, sp.xt)
            sp.v[:, 0] += (d["q"][s] / d["m"][s]) * Ep * dt
            sp.xt = sp.xt + sp.v[:, 0] * dt / dx
            if record:
                rec[f"pushed_id_{s}"] = sp.id.copy()
                rec[f"pushed_xt_{s}"] = sp.xt.copy()
            # 5. walls
            lost = (sp.xt < 0) | (sp.xt >= N)
            self._wall(s, lost, rec if record else None)
            if lost.any():
                sp.take(~lost)
            # 6. Monte Carlo collisions at x^(l+1)
            due = sp.next == l
            cand = np.nonzero(due & ~sp.redraw)[0]
            a["candidates"][s] += cand.size
            if record:
                rec[f"cand_id_{s}"] = sp.id[cand].copy()
            re = np.nonzero(due & sp.redraw)[0]
            a["redraws"][s] += re.size
            if re.size:
                # a cut wait: a fresh wait from the candidate draw's U7
                U = R.draw(sp.id[re], l, R.tag(s, R.COLL), p["seed"], p["case_id"])
                sp.next[re], sp.redraw[re], rtie = skip(U[:, 7], l, d["p_tot"][s], self.wait_cap)
                if record:
                    rec[f"redraw_id_{s}"] = sp.id[re].copy()
                    rec[f"redraw_tie_{s}"] = rtie
            if cand.size:
                births.extend(self._mcc(s, cand, l, rec if record else None))
            if record:
                rec[f"xt_{s}"] = sp.xt.copy()
                rec[f"v_{s}"] = sp.v.copy()
                rec[f"id_{s}"] = sp.id.copy()
                rec[f"next_{s}"] = sp.next.copy()
                rec[f"redraw_{s}"] = sp.redraw.copy()
        for (s, xt, v, ids, nxt, rd) in births:
            self.sp[s].append(xt, v, ids, nxt, rd)
            a["births"] += ids.size
        cap = (p.get("capacity_e", 1 << 62), p.get("capacity_i", 1 << 62))
        if len(self.sp[0]) > cap[0] or len(self.sp[1]) > cap[1]:
            self.status = ECAPACITY
        self.step_index = l + 1
        return rec

    def _wall(self, s, lost, rec):
        """Absorbing electrodes; ions record impact energy and angle."""
        a, sp = self.acc, self.sp[s]
        left = lost & (sp.xt < 0)
        right = lost & ~(sp.xt < 0)
        a["absorbed"][s, 0] += int(np.count_nonzero(left))
        a["absorbed"][s, 1] += int(np.count_nonzero(right))
        self.n_abs_net += (1 if s == 1 else -1) * int(np.count_nonzero(left))
        if rec is not None:
            rec[f"lost_id_{s}"] = sp.id[lost].copy()
            rec[f"lost_left_{s}"] = left[lost].copy()
        if s == 1 and np.any(lost):
            v = sp.v[lost]
            speed2 = np.sum(v * v, axis=1)
            E_ev = 0.5 * C.M_AR * speed2 / C.E_CHARGE
            theta = np.degrees(np.arccos(np.minimum(np.abs(v[:, 0]) / np.sqrt(speed2), 1.0)))
            el = np.where(left[lost], 0, 1)
            eb = np.minimum(np.floor(E_ev).astype(np.int64), self.d["n_ebins"] - 1)
            ab = np.minimum(np.floor(theta / ANGLE_BIN_DEG).astype(np.int64), N_ANGLE_BINS - 1)
            np.add.at(a["iedf"], (el, eb), 1)
            np.add.at(a["iadf"], (el, ab), 1)
            np.add.at(a["iead"], (el, eb // IEAD_E_GROUP, ab // IEAD_A_GROUP), 1)
            np.add.at(a["ion_energy_sum"], el, E_ev)
            if rec is not None:
                rec["lost_ion_E"] = E_ev
                rec["lost_ion_theta"] = theta

    def _mcc(self, s, idx, l, rec):
        """Null-collision Monte Carlo collisions of the candidates ``idx`` at step l."""
        p, d, a = self.p, self.d, self.acc
        sp = self.sp[s]
        key = (p["seed"], p["case_id"])
        ids = sp.id[idx]
        v = sp.v[idx]
        m, M = d["m"][s], C.M_AR
        mr = d["mr"][s]
        nu_max = d["nu_max"][s]
        n_gas = d["n_gas"]
        # all random numbers of a candidate come from one draw: U0 selects the
        # process, U1-U2 (and U3-U4 for ionisation) the electron directions or
        # U1-U4 the ion's Maxwellian partner, U7 the waiting time to its next
        # candidate
        U = R.draw(ids, l, R.tag(s, R.COLL), *key)
        birth = []
        if s == 0:
            g = v                                   # gas at rest for electrons
            g2 = np.sum(g * g, axis=1)
            gm = np.sqrt(g2)
            eps = 0.5 * mr * g2 / C.E_CHARGE
            s_el, s_exc, s_ion = electron_sigmas(eps, p)
            S1 = n_gas * s_el * gm
            S2 = S1 + n_gas * s_exc * gm
            S3 = S2 + n_gas * s_ion * gm
            r = U[:, 0] * nu_max
            proc = np.where(r < S1, P_EL, np.where(r < S2, P_EXC, np.where(r < S3, P_ION, P_NULL)))
            tie = np.min(np.abs(np.stack([r - S1, r - S2, r - S3])), axis=0) < 2.0 ** -20 * nu_max
            a["overflow"][0] += int(np.count_nonzero(S3 > nu_max))
            for j in (P_EL, P_EXC, P_ION):
                a["collisions"][j] += int(np.count_nonzero(proc == j))
            vnew = v.copy()
            # elastic and excitation: isotropic in the CM frame, target at rest
            nhat = isotropic_direction(U[:, 1], U[:, 2])
            Vcm = (m / (m + M)) * v
            sc = (proc == P_EL) | (proc == P_EXC)
            gp = np.where(proc == P_EXC,
                          np.sqrt(np.maximum(g2 - 2.0 * p["eth_exc"] * C.E_CHARGE / mr, 0.0)), gm)
            vs = Vcm + (M / (m + M)) * gp[:, None] * nhat
            vnew[sc] = vs[sc]
            # ionisation: two electrons with (eps - E_ion)/2 each, new Maxwellian ion
            io = np.nonzero(proc == P_ION)[0]
            if io.size:
                Ek = np.maximum(0.5 * (eps[io] - p["eth_ion"]), 0.0)
                speed = np.sqrt(2.0 * Ek * C.E_CHARGE / C.M_E)
                vnew[io] = speed[:, None] * isotropic_direction(U[io, 1], U[io, 2])
                v2 = speed[:, None] * isotropic_direction(U[io, 3], U[io, 4])
                pid = ids[io]
                Ui = R.draw(pid, l, R.tag(0, R.ION), *key)
                vion = R.maxwell_velocity(Ui[:, 0:4], math.sqrt(C.K_B * p["t_gas_k"] / C.M_AR))
                w0, w1, _, _ = R.philox4x64(pid, np.uint64(l), R.tag(0, R.CHILD), 0, *key)
                xt_c = sp.xt[idx[io]]
                Ue = R.draw(w0, l, R.tag(0, R.SKIP), *key)
                Ui2 = R.draw(w1, l, R.tag(1, R.SKIP), *key)
                ne, re_e, _ = skip(Ue[:, 0], l, d["p_tot"][0], self.wait_cap)
                ni, re_i, _ = skip(Ui2[:, 0], l, d["p_tot"][1], self.wait_cap)
                birth = [(0, xt_c.copy(), v2, w0, ne, re_e), (1, xt_c.copy(), vion, w1, ni, re_i)]
                if rec is not None:
                    rec["birth_e"] = (w0, xt_c.copy(), v2.copy(), ne)
                    rec["birth_i"] = (w1, xt_c.copy(), vion.copy(), ni)
            sp.v[idx] = vnew
        else:
            vbg = R.maxwell_velocity(U[:, 1:5], math.sqrt(C.K_B * p["t_gas_k"] / C.M_AR))
            g = v - vbg
            gm = np.sqrt(np.sum(g * g, axis=1))
            S1 = n_gas * p["sigma_cx"] * gm
            r = U[:, 0] * nu_max
            proc = np.where(r < S1, P_CX, P_NULL)
            tie = np.abs(r - S1) < 2.0 ** -20 * nu_max
            a["overflow"][1] += int(np.count_nonzero(S1 > nu_max))
            a["collisions"][4] += int(np.count_nonzero(proc == P_CX))
            cx = proc == P_CX
            vnew = v.copy()
            vnew[cx] = vbg[cx]                       # resonant charge exchange
            sp.v[idx] = vnew
        # next candidate of every candidate particle
        sp.next[idx], sp.redraw[idx], skip_tie = skip(U[:, 7], l, d["p_tot"][s], self.wait_cap)
        if rec is not None:
            rec[f"proc_{s}"] = proc
            rec[f"tie_{s}"] = tie
            rec[f"skip_tie_{s}"] = skip_tie
        # births are appended by the caller after both species were advanced
        return birth

    def run(self, n_steps):
        for _ in range(n_steps):
            self.step()
