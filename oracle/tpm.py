"""FP64 oracle of the test-particle method for sputtered atoms (Sec. IV.B).

Source ('Wall Interactions'): every ion hitting the target is checked N = ceil(Y)
times with R_f <= Y / N, each success emitting one atom at the impact point
(x = 0).  Each atom's energy follows the Sigmund-Thompson flux distribution
f(E) ~ E / (E + U_s)^3 truncated at E_cut, its polar angle the cosine law
theta = arccos(sqrt(R_f)), its azimuth psi = 2 pi R_f.  The energy is drawn by
inverting the truncated CDF, (E/(E+U_s))^2 / s_max^2 with s_max =
E_cut/(E_cut+U_s): same law as the acceptance-rejection sampling the paper
mentions, with a fixed number of draws.

Flight ('Collisional Transport', 'Binary Interactions', Eq. (5)): straight
flights between candidate events whose times follow tau = -tau_c ln R_f with
tau_c = 1/nu_max, nu_max = n_bg (sigma v_r)_max (the null-collision majorant of
Eq. (6) applied to the test species).  At each candidate a background partner is
drawn from the Maxwellian gas; the event is a real collision with probability
sigma(v_r) v_r / (sigma v_r)_max, where sigma = pi b_max^2 and b_max follows
Eq. (8) (variable hard sphere).  A real collision scatters isotropically in the
centre-of-mass frame (impact parameter b = b_max sqrt(R_f), chi = 2 arccos(b /
b_max), psi = 2 pi R_f; Eq. (10) and the VHS law).  The flight time is the
gridless time step of the paper's closing TPM paragraph (dt equal to the time
to the next candidate event).

M1 scattering (``scatter`` = SCATTER_M1; 'Binary Interactions', the modified
VHS model): the deflection is chi = pi (1 - b / b_max) with b = b_max sqrt(R_f),
about the pre-collision relative velocity, at azimuth psi = 2 pi R_f, and the
VHS cross section is used with the reference diameter sqrt(4/3) d_ref.  The
post-collision relative velocity is the pre-collision one turned by (chi, psi)
(the coordinate transform the paper cites; rotate_relative below).

Fixed time step (``dt_s`` > 0; 'Collisional Transport', Eq. (7)): every flight
lasts dt and is followed by a collision test with the linearised probability
P = n_bg sigma(v_r) v_r dt for a freshly drawn partner (a real collision when
R_f < P; P > 1 is counted as an overflow).  With dt the PIC step the atoms
share the plasma's clock.  The gridless flight above is dt_s = 0.

Walls: atoms that reach x < 0 (target) or x >= L (substrate) stick (perfect
sinks) and are tallied.  The lateral directions are periodic.

Readings: (sigma v_r)_max is evaluated at g_cap = v(E_cut) + 10 sqrt(k_B T /
m_gas); faster pairs are accepted and counted as overflows.  An atom still in
flight after ``e_max`` candidate events is counted as unfinished.

Spatial profiles (the sputtered-atom density and mean velocity of the results
section): track-length tallies on ``n_xbins`` equal cells of the gap.  Every
straight flight from x_a to x_b adds to each cell the time it spends there,
overlap / |v_x|, and its signed x-displacement there, overlap * sign(v_x).
With the source flux Gamma (m^-2 s^-1) the density of a cell is
Gamma / n_atoms * time / dx and the mean x-velocity displacement / time.
"""
import math
import numpy as np

from . import constants as C
from . import philox as R
from .xsec import vhs_sigma
from .pic import isotropic_direction

MODE_NORMAL, MODE_BOX = 0, 1
SCATTER_VHS, SCATTER_M1 = 0, 1
WALL_TARGET, WALL_SUBSTRATE, UNFINISHED = 0, 1, 2
N_THETA_BINS = 90                         # 1 degree bins


def masses(tp):
    """(m_test, m_gas) in kg from the atomic masses of the flight parameters."""
    return tp["m_test_amu"] * C.AMU, tp["m_gas_amu"] * C.AMU


def thompson_energy(U, u_s, e_cut):
    """Sigmund-Thompson flux energy by inversion of the truncated CDF."""
    s_max = e_cut / (e_cut + u_s)
    s = np.sqrt(U) * s_max
    return u_s * s / (1.0 - s)


def source(n_atoms, src, tp, first_id=0):
    """Initial state of atoms first_id .. first_id + n_atoms - 1 (x, y, z, v).
    ``electrode`` 0 emits from the target (x = 0, into +x); 1 from the substrate
    (x = L, into -x): re-sputtering of the Al-coated substrate by its own ion
    impacts (results section), the mirror image of the target's emission."""
    ids = np.arange(first_id, first_id + n_atoms, dtype=np.uint64)
    U = R.draw(ids, 0, R.tag(R.SP_AL, R.TP_SRC), src["seed"], src["job_id"])
    E = thompson_energy(U[:, 0], src["u_s_ev"], src["e_cut_ev"])
    theta = np.arccos(np.sqrt(U[:, 1]))
    psi = 2.0 * np.pi * U[:, 2]
    speed = np.sqrt(2.0 * E * C.E_CHARGE / masses(tp)[0])
    v = speed[:, None] * np.stack([np.cos(theta), np.sin(theta) * np.cos(psi),
                                   np.sin(theta) * np.sin(psi)], axis=-1)
    pos = np.zeros((n_atoms, 3))
    if src.get("electrode", 0) == 1:
        pos[:, 0] = tp["gap_m"]
        v[:, 0] = -v[:, 0]
    pos[:, 1] = tp["lateral_m"] * U[:, 3]
    pos[:, 2] = tp["lateral_m"] * U[:, 4]
    return ids, pos, v, E


def d_ref_of(tp):
    """The reference diameter of the scattering law: d_ref for VHS, sqrt(4/3) d_ref
    for M1 (the VHS data reused for M1, 'Binary Interactions')."""
    return tp["d_ref"] * (math.sqrt(4.0 / 3.0) if tp.get("scatter", SCATTER_VHS) == SCATTER_M1 else 1.0)


def rotate_relative(g, chi, psi):
    """The relative velocity g (rows) turned by the deflection chi at azimuth psi
    about its own direction: |g'| = |g|, angle(g, g') = chi.  The azimuth is
    measured in the plane normal to g from the direction e1 = (x-hat x g) / |.|
    (from e1 = y-hat when g lies within 1e-6 of the x axis)."""
    gm = np.linalg.norm(g, axis=1)
    ghat = g / gm[:, None]
    e1 = np.stack([np.zeros_like(gm), -ghat[:, 2], ghat[:, 1]], axis=1)
    n1 = np.linalg.norm(e1, axis=1)
    along = n1 <= 1e-6
    e1[along] = np.array([0.0, 1.0, 0.0])
    e1[~along] /= n1[~along, None]
    e2 = np.cross(ghat, e1)
    d = (np.cos(chi)[:, None] * ghat
         + (np.sin(chi) * np.cos(psi))[:, None] * e1 + (np.sin(chi) * np.sin(psi))[:, None] * e2)
    return gm[:, None] * d


def scatter(v, vbg, Ua, Ub, m, M, law):
    """Post-collision velocity of the test atom (v) after a real collision with the
    gas partner vbg: the centre-of-mass velocity plus M/(m+M) times the new relative
    velocity, drawn from Ua, Ub -- isotropic for VHS (Eq. (10) with the VHS law),
    or g turned by chi = pi (1 - sqrt(Ua)) at psi = 2 pi Ub for M1."""
    Vcm = (m * v + M * vbg) / (m + M)
    g = v - vbg
    if law == SCATTER_M1:
        return Vcm + (M / (m + M)) * rotate_relative(g, np.pi * (1.0 - np.sqrt(Ua)), 2.0 * np.pi * Ub)
    gm = np.sqrt(np.sum(g * g, axis=1))
    nhat = isotropic_direction(Ua, Ub)
    return Vcm + (M / (m + M)) * gm[:, None] * nhat


def collision_probability(n_gas, sg, dt):
    """Eq. (7): the linearised probability of a collision within dt with a
    partner at relative speed g, P = n_bg sigma(g) g dt (sg = sigma(g) g)."""
    return n_gas * sg * dt


def majorant(src, tp):
    """(sigma v_r)_max at the capped relative speed and nu_max = n_bg times it."""
    m, M = masses(tp)
    mr = m * M / (m + M)
    g_cap = math.sqrt(2.0 * src["e_cut_ev"] * C.E_CHARGE / m) + 10.0 * math.sqrt(C.K_B * tp["t_gas_k"] / M)
    sg_max = float(vhs_sigma(g_cap, mr, d_ref_of(tp), tp["omega"], tp["t_ref"])) * g_cap
    n_gas = C.gas_density(tp["p_pa"], tp["t_gas_k"])
    return sg_max, n_gas * sg_max


def run(src, tp, n_atoms=None, first_id=0, trace=False):
    """Fly atoms first_id .. first_id + n_atoms - 1 to a wall; returns tallies
    (and, with ``trace``, one record per atom)."""
    n_atoms = int(src["n_atoms"] if n_atoms is None else n_atoms)
    m, M = masses(tp)
    mr = m * M / (m + M)
    L, lat = tp["gap_m"], tp["lateral_m"]
    sg_max, nu_max = majorant(src, tp)
    sig_gas = math.sqrt(C.K_B * tp["t_gas_k"] / M)
    key = (src["seed"], src["job_id"])
    ids, pos, v, E0 = source(n_atoms, src, tp, first_id)
    t = np.zeros(n_atoms)
    nev = np.zeros(n_atoms, dtype=np.int64)
    wall = np.full(n_atoms, UNFINISHED, dtype=np.int64)
    t_hit = np.zeros(n_atoms)
    v_hit = np.zeros((n_atoms, 3))
    n_coll = 0
    n_over = 0
    e_max = int(tp["e_max"])
    n_x = int(tp.get("n_xbins", 0)) if tp["mode"] == MODE_NORMAL else 0
    time_s, disp_m = np.zeros(n_x), np.zeros(n_x)
    active = np.arange(n_atoms)
    dt_fixed = float(tp.get("dt_s", 0.0))
    n_gas = C.gas_density(tp["p_pa"], tp["t_gas_k"])
    while active.size:
        U = R.draw(ids[active], nev[active], R.tag(R.SP_AL, R.TP_EVT), *key)
        if dt_fixed > 0.0:
            tau = np.full(active.size, dt_fixed)
        else:
            with np.errstate(divide="ignore"):
                tau = -np.log(U[:, 0]) / nu_max if nu_max > 0 else np.full(active.size, np.inf)
        x, vx = pos[active, 0], v[active, 0]
        with np.errstate(invalid="ignore"):
            xn = x + vx * tau
        if tp["mode"] == MODE_NORMAL:
            sub = xn >= L
            tgt = xn < 0
            hit = sub | tgt
            with np.errstate(divide="ignore", invalid="ignore"):
                dt_hit = np.where(sub, (L - x) / vx, -x / vx)
            h = active[hit]
            wall[h] = np.where(sub[hit], WALL_SUBSTRATE, WALL_TARGET)
            t_hit[h] = t[h] + dt_hit[hit]
            v_hit[h] = v[h]
            if n_x:
                track_tally(time_s, disp_m, x[hit], np.where(sub[hit], L, 0.0), vx[hit], n_x, L)
                track_tally(time_s, disp_m, x[~hit], xn[~hit], vx[~hit], n_x, L)
        else:
            hit = np.zeros(active.size, dtype=bool)
            xn = np.mod(xn, L)
        go = active[~hit]
        tg = tau[~hit]
        Ug = U[~hit]
        pos[go, 0] = xn[~hit]
        pos[go, 1:] = np.mod(pos[go, 1:] + v[go, 1:] * tg[:, None], lat)
        t[go] += tg
        # candidate event: Maxwellian partner and acceptance sigma g / (sigma g)_max
        vbg = R.maxwell_velocity(Ug[:, 1:5], sig_gas)
        g = v[go] - vbg
        gm = np.sqrt(np.sum(g * g, axis=1))
        sg = vhs_sigma(gm, mr, d_ref_of(tp), tp["omega"], tp["t_ref"]) * gm
        if dt_fixed > 0.0:
            P_c = collision_probability(n_gas, sg, dt_fixed)
            n_over += int(np.count_nonzero(P_c > 1.0))
            acc = Ug[:, 5] < P_c
        else:
            n_over += int(np.count_nonzero(sg > sg_max))
            acc = Ug[:, 5] * sg_max < sg
        n_coll += int(np.count_nonzero(acc))
        a = go[acc]
        v[a] = scatter(v[a], vbg[acc], Ug[acc, 6], Ug[acc, 7], m, M, tp.get("scatter", SCATTER_VHS))
        nev[go] += 1
        done = nev[go] >= e_max
        unf = go[done]
        v_hit[unf] = v[unf]
        t_hit[unf] = t[unf]
        active = go[~done]

    speed2 = np.sum(v_hit * v_hit, axis=1)
    E_hit = 0.5 * m * speed2 / C.E_CHARGE
    with np.errstate(invalid="ignore", divide="ignore"):
        theta = np.degrees(np.arccos(np.minimum(np.abs(v_hit[:, 0]) / np.sqrt(speed2), 1.0)))
    res = tally(wall, E_hit, theta, t_hit, tp)
    res.update(n_atoms=n_atoms, events=int(nev.sum()), collisions=n_coll, overflow=n_over,
               nu_max=nu_max, sg_max=sg_max)
    if n_x:
        res.update(time_s=time_s, disp_m=disp_m)
        res["density_m3"], res["mean_vx"] = profiles(res, src, n_atoms, L)
    if trace:
        res["trace"] = dict(id=ids, wall=wall, events=nev, E=E_hit, theta=theta, tof=t_hit,
                            v=v_hit, E0=E0, x=pos[:, 0].copy())
    return res


def cell_overlaps(xa, xb, n_bins, L):
    """Length of each flight [min(xa, xb), max(xa, xb)] inside each of n_bins
    equal cells of [0, L): an array (flights x cells)."""
    lo = np.minimum(xa, xb)[:, None]
    hi = np.maximum(xa, xb)[:, None]
    edges = np.arange(n_bins + 1) * (L / n_bins)
    return np.clip(np.minimum(hi, edges[None, 1:]) - np.maximum(lo, edges[None, :-1]), 0.0, None)


def track_tally(time_s, disp_m, xa, xb, vx, n_bins, L):
    """Add the residence time and signed x-displacement of flights xa -> xb."""
    if xa.size == 0:
        return
    ov = cell_overlaps(xa, xb, n_bins, L)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(vx != 0, 1.0 / np.abs(vx), 0.0)
    time_s += (ov * inv[:, None]).sum(axis=0)
    disp_m += (ov * np.sign(vx)[:, None]).sum(axis=0)


def profiles(res, src, n_atoms, L):
    """Density (m^-3) and mean x-velocity (m/s) per cell from the tallies."""
    n_bins = res["time_s"].size
    dx = L / n_bins
    flux = float(src.get("flux_m2s", 0.0))
    dens = flux / max(n_atoms, 1) * res["time_s"] / dx
    with np.errstate(divide="ignore", invalid="ignore"):
        ux = np.where(res["time_s"] > 0, res["disp_m"] / res["time_s"], 0.0)
    return dens, ux


def tally(wall, E, theta, tof, tp):
    """Counts and histograms of the atoms absorbed at the substrate and target."""
    sub = wall == WALL_SUBSTRATE
    nb, eb = int(tp["n_ebins"]), float(tp["ebin_ev"])
    ntb, tb = int(tp["n_tbins"]), float(tp["tbin_s"])
    Es, ths, ts = E[sub], theta[sub], tof[sub]
    e_hist = np.bincount(np.minimum(np.floor(Es / eb).astype(np.int64), nb - 1), minlength=nb)
    a_hist = np.bincount(np.minimum(np.floor(ths).astype(np.int64), N_THETA_BINS - 1), minlength=N_THETA_BINS)
    t_hist = np.bincount(np.minimum(np.floor(ts / tb).astype(np.int64), ntb - 1), minlength=ntb)
    return dict(n_substrate=int(sub.sum()), n_target=int((wall == WALL_TARGET).sum()),
                n_unfinished=int((wall == UNFINISHED).sum()),
                e_hist=e_hist, theta_hist=a_hist, tof_hist=t_hist,
                e_sum_substrate=float(Es.sum()), e_sum_target=float(E[wall == WALL_TARGET].sum()))


def yield_of(E_ev, yld):
    """Sputter yield Y(E): a constant, or linear interpolation in a table."""
    if np.isscalar(yld) or np.ndim(yld) == 0:
        return np.full(np.shape(E_ev), float(yld))
    Et, Yt = np.asarray(yld[0], dtype=float), np.asarray(yld[1], dtype=float)
    return np.interp(E_ev, Et, Yt)


def sputtered_count(iedf_target, yld, seed, job_id, ebin_ev=1.0, electrode=0, taken=None):
    """Number of atoms emitted by the recorded ion impacts on one electrode
    ('Wall Interactions' of Sec. IV.B): each impact in energy bin b (energy taken
    at the bin centre) makes N = ceil(Y) checks R_f <= Y / N.  The draws of
    electrode e use aux = e 2^32 + check index; impact i of bin b is keyed by
    (i, b), so ``taken`` (impacts of each bin already turned into atoms) selects
    the impacts i >= taken[b] that arrived since: counting in pieces as the
    impacts arrive draws exactly what one count of the whole record draws."""
    emitted = 0
    iedf = np.asarray(iedf_target, dtype=np.int64)
    t0 = np.zeros_like(iedf) if taken is None else np.asarray(taken, dtype=np.int64)
    for b, c in enumerate(iedf):
        if c <= t0[b]:
            continue
        Y = float(yield_of((b + 0.5) * ebin_ev, yld))
        N = int(math.ceil(Y))
        if N == 0:
            continue
        p = Y / N
        i = np.repeat(np.arange(t0[b], c, dtype=np.uint64), N)
        n = np.tile(np.arange(N, dtype=np.uint64), int(c - t0[b]))
        U = R.draw(i, b, R.tag(R.SP_YIELD, R.YIELD), seed, job_id, aux=n + (np.uint64(electrode) << np.uint64(32)))
        emitted += int(np.count_nonzero(U[:, 0] <= p))
    return emitted
