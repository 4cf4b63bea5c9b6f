"""Pins of the PIC/MCC oracle against closed forms, library routines and the
paper's printed value.  Each check raises AssertionError on failure; the
``test_oracle_*`` modules run them, and ``test_oracle_mutations`` plants mistakes
in the oracle to show that the checks catch them.
"""
import math
from fractions import Fraction

import numpy as np
from scipy import stats

from oracle import constants as C
from oracle import philox as R
from oracle import pic as P
from oracle.xsec import electron_sigmas
import workloads as W


def field_free_case(**kw):
    p = W.discharge_small()
    p.update(flags=P.NO_SELF_FIELD | P.NO_COLLISIONS)
    p.update(kw)
    return p


# ----------------------------------------------------------------- charge
def check_deposit_exact(seed=0):
    N = 16
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0, N, 257)
    xt[:4] = [3.0, 2.25, 0.0, N - 2.0 ** -40]
    Q = P.deposit(xt, N)
    assert Q.sum() == xt.size * 2 ** 32                       # each particle deposits 2^32
    # brute force with exact rationals: frac * 2^32 rounded half-to-even
    B = [0] * (N + 1)
    for x in xt:
        fx = Fraction(float(x))
        j = math.floor(fx)
        Wt = round((fx - j) * 2 ** 32)
        B[j] += 2 ** 32 - Wt
        B[j + 1] += Wt
    assert list(Q) == B
    one = P.deposit(np.array([2.25]), N)
    assert one[2] == 3 * 2 ** 30 and one[3] == 2 ** 30 and one.sum() == 2 ** 32
    node = P.deposit(np.array([3.0]), N)
    assert node[3] == 2 ** 32 and node.sum() == 2 ** 32
    perm = rng.permutation(xt.size)
    assert np.array_equal(P.deposit(xt[perm], N), Q)


# ------------------------------------------------------------------ field
def check_poisson_uniform_rho_exact(N=64, L=0.025, V=137.0, q=12345 * 2 ** 20, w=5e9):
    """Uniform rho0 with Phi_0 = V, Phi_N = 0: the FD solution equals the parabola
    V (1 - x/L) + rho0 x (L - x) / (2 eps0) at the nodes, and E (with the half-cell
    boundary reading) equals -dPhi/dx of the parabola at every node."""
    dx = L / N
    Qi = np.full(N + 1, q, dtype=np.int64)
    Qi[0] = Qi[N] = q // 2
    Qe = np.zeros(N + 1, dtype=np.int64)
    rho = P.charge_density(Qe, Qi, w, dx, N)
    rho0 = C.E_CHARGE * w * q / (2 ** 32 * dx)
    assert np.allclose(rho, rho0, rtol=1e-15, atol=0)
    x = np.arange(N + 1) * dx
    Phi = P.solve_potential(rho, V, dx)
    Phi_exact = V * (1 - x / L) + rho0 * x * (L - x) / (2 * C.EPS0)
    scale = np.max(np.abs(Phi_exact))
    assert np.max(np.abs(Phi - Phi_exact)) <= 1e-12 * scale
    E = P.electric_field(Phi, rho, dx)
    E_exact = V / L - rho0 * (L - 2 * x) / (2 * C.EPS0)
    assert np.max(np.abs(E - E_exact)) <= 1e-10 * np.max(np.abs(E_exact))


def check_poisson_random_vs_dense(seed=1, N=50):
    """Random charge: the banded solve equals a dense LAPACK solve of the full
    (N+1) x (N+1) system with Dirichlet rows."""
    rng = np.random.default_rng(seed)
    dx = 1e-4
    rho = rng.normal(size=N + 1) * 1e-6
    V = -42.0
    A = np.zeros((N + 1, N + 1))
    b = np.zeros(N + 1)
    A[0, 0] = 1.0
    b[0] = V
    A[N, N] = 1.0
    for m in range(1, N):
        A[m, m - 1], A[m, m], A[m, m + 1] = 1.0, -2.0, 1.0
        b[m] = -rho[m] * dx * dx / C.EPS0
    ref = np.linalg.solve(A, b)
    Phi = P.solve_potential(rho, V, dx)
    assert np.max(np.abs(Phi - ref)) <= 1e-12 * np.max(np.abs(ref))
    E = P.electric_field(Phi, rho, dx)
    assert np.allclose(E[1:N], -(ref[2:] - ref[:-2]) / (2 * dx), rtol=1e-9, atol=1e-9 * np.max(np.abs(E)))


def check_gather_linear_exact(seed=2, N=32):
    rng = np.random.default_rng(seed)
    a, b = 3.5, -0.75
    E = a + b * np.arange(N + 1)
    xt = rng.uniform(0, N, 1000)
    assert np.allclose(P.gather(E, xt), a + b * xt, rtol=0, atol=1e-12)


# ------------------------------------------------------------------- push
def _static_field_case(V=1e-3):
    # one step per "cycle" makes V(t_l) = V0 cos(phi) the same at every step
    return field_free_case(v0_volt=V, phase_rad=0.0, steps_per_cycle=1, freq_hz=1e10, p_pa=1.0)


def _set_state(d, s, xt, v):
    sp = d.sp[s]
    n = xt.size
    sp.xt = np.array(xt, dtype=np.float64)
    sp.v = np.array(v, dtype=np.float64)
    sp.id = np.arange(n, dtype=np.uint64)
    sp.next = np.full(n, P.NEVER, dtype=np.int64)
    sp.redraw = np.zeros(n, dtype=bool)


def check_uniform_field_trajectory(n_steps=100):
    """Static uniform field: leapfrog reproduces x^(l) = x0 + l dt v^(-1/2)
    + a dt^2 l (l+1) / 2 exactly (it integrates constant acceleration exactly)."""
    p = _static_field_case()
    d = P.Discharge(p, load=False)
    L, dx, dt, N = p["gap_m"], d.d["dx"], d.d["dt"], d.d["N"]
    rng = np.random.default_rng(3)
    n = 64
    xt0 = rng.uniform(0.4 * N, 0.6 * N, n)
    v0 = np.zeros((n, 3))
    v0[:, 0] = rng.normal(0, 1e4, n)
    for s in (0, 1):
        _set_state(d, s, xt0, v0)
    E = p["v0_volt"] / L
    for l in range(1, n_steps + 1):
        d.step()
        for s in (0, 1):
            a = d.d["q"][s] * E / d.d["m"][s]
            x = xt0 * dx + l * dt * v0[:, 0] + a * dt * dt * l * (l + 1) / 2
            assert np.allclose(d.sp[s].xt * dx, x, rtol=1e-12, atol=1e-15)


def check_time_centred_energy_conserved(n_steps=200):
    """Static uniform field: 0.5 m v^(l-1/2) v^(l+1/2) + q Phi(x^(l)) is exactly
    conserved by the leapfrog scheme."""
    p = _static_field_case(V=5e-3)
    d = P.Discharge(p, load=False)
    L, dx, N = p["gap_m"], d.d["dx"], d.d["N"]
    rng = np.random.default_rng(4)
    n = 64
    xt0 = rng.uniform(0.45 * N, 0.55 * N, n)
    v0 = np.zeros((n, 3))
    v0[:, 0] = rng.normal(0, 3e3, n)
    _set_state(d, 0, xt0, v0)
    _set_state(d, 1, xt0[:0], v0[:0])
    V = p["v0_volt"]
    m, q = d.d["m"][0], d.d["q"][0]
    prev_v = v0[:, 0].copy()
    prev_x = xt0 * dx
    ref = None
    for _ in range(n_steps):
        d.step()
        v = d.sp[0].v[:, 0]
        Et = 0.5 * m * prev_v * v + q * V * (1 - prev_x / L)
        if ref is None:
            ref = Et
        assert np.allclose(Et, ref, rtol=1e-9, atol=1e-12 * np.max(np.abs(ref)))
        prev_v = v.copy()
        prev_x = d.sp[0].xt * dx


# ------------------------------------------------------------- collisions
def check_ionisation_peak():
    """sigma0 ln(x)/x peaks at x = e with value sigma0/e (42.95 eV for 15.8 eV)."""
    xs = W.XSEC
    eps = np.linspace(16, 200, 200001)
    s = electron_sigmas(eps, xs)[2]
    k = np.argmax(s)
    assert abs(eps[k] - 15.8 * math.e) < 2e-3
    assert abs(s[k] - 2.5e-20 / math.e) < 1e-27


def check_null_collision_selection(energy_ev=60.0, n=400000):
    """Given a candidate, process j is selected with probability nu_j(eps)/nu_max
    and the null process with the rest (Eq. (6) and the selection rule)."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0)
    d = P.Discharge(p, load=False)
    N = d.d["N"]
    mr = d.d["mr"][0]
    rng = np.random.default_rng(5)
    g = math.sqrt(2 * energy_ev * C.E_CHARGE / mr)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    # no field: the push keeps v, so every electron meets step 0's check at energy eps
    _set_state(d, 0, np.full(n, N / 2 + 0.25), g * dirs)
    _set_state(d, 1, np.zeros(0), np.zeros((0, 3)))
    d.sp[0].next[:] = 0
    rec = d.step(record=True)
    proc = rec["proc_0"]
    n_gas, nu_max = d.d["n_gas"], d.d["nu_max"][0]
    sig = electron_sigmas(np.array([energy_ev]), W.XSEC)
    frac = [n_gas * s[0] * g / nu_max for s in sig]
    for j in (P.P_EL, P.P_EXC, P.P_ION):
        k = int(np.count_nonzero(proc == j))
        lo, hi = stats.binom.interval(1 - 1e-6, n, frac[j])
        assert lo <= k <= hi, (j, k, n * frac[j])
    assert d.acc["births"] == 2 * int(np.count_nonzero(proc == P.P_ION))   # e + Ar+ per event


def check_first_collision_law(energy_ev=60.0, n=100000, steps=40):
    """The schedule and the selection together, over many steps: electrons of one
    energy, moving parallel to the electrodes in a field-free gap (so they keep
    their energy and position until they collide), each with its first wait
    drawn as at a load.  The per-step hazard of a first real collision must be
    P_tot nu_T / nu_max exactly (independent per-step checks, Eq. (6) with the
    selection rule), and within O(nu_max dt) of the direct per-process law
    1 - exp(-nu_T dt) of a Poisson collision process."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0)
    d = P.Discharge(p, load=False)
    N, dt = d.d["N"], d.d["dt"]
    mr = d.d["mr"][0]
    g = math.sqrt(2 * energy_ev * C.E_CHARGE / mr)
    phi = np.random.default_rng(8).uniform(0.0, 2 * np.pi, n)
    _set_state(d, 0, np.full(n, N / 2 + 0.25), g * np.stack([np.zeros(n), np.cos(phi), np.sin(phi)], axis=1))
    _set_state(d, 1, np.zeros(0), np.zeros((0, 3)))
    p_tot = d.d["p_tot"][0]
    Us = R.draw(d.sp[0].id, np.uint64(2 ** 64 - 1), R.tag(0, R.SKIP), p["seed"], p["case_id"])
    d.sp[0].next, d.sp[0].redraw, _ = P.skip(Us[:, 0], -1, p_tot)
    first = np.full(n, -1)
    for l in range(steps):
        rec = d.step(record=True)
        cid = rec.get("cand_id_0", np.zeros(0, np.uint64))
        proc = rec.get("proc_0", np.zeros(0, int))
        hit = cid[(proc != P.P_NULL) & (cid < n)].astype(np.int64)
        hit = hit[first[hit] < 0]
        first[hit] = l
    at_risk = np.array([np.count_nonzero((first < 0) | (first >= l)) for l in range(steps)])
    events = np.bincount(first[first >= 0], minlength=steps)
    X, E = int(at_risk.sum()), int(events.sum())
    sig = electron_sigmas(np.array([energy_ev]), W.XSEC)
    nu_t = d.d["n_gas"] * sum(float(s_[0]) for s_ in sig) * g
    nu_max = d.d["nu_max"][0]
    h = p_tot * nu_t / nu_max
    sd = math.sqrt(X * h * (1 - h))
    assert abs(E - X * h) <= 5 * sd, (E, X * h, sd)
    h_direct = -math.expm1(-nu_t * dt)
    assert abs(h - h_direct) <= nu_t * dt * nu_max * dt, (h, h_direct)
    assert abs(E / X - h_direct) <= 5 * sd / X + nu_t * dt * nu_max * dt


def check_skip_law(p_tot=0.0123, n=400000):
    """The geometric waiting time has the law of independent per-step checks
    R_f <= P_c,tot: P(G = k) = (1 - P)^(k-1) P."""
    ids = np.arange(n, dtype=np.uint64)
    U = R.draw(ids, 77, R.tag(0, R.SKIP), 5, 6)
    nxt, redraw, _ = P.skip(U[:, 0], 10, p_tot)
    assert not redraw.any()
    G = nxt - 10
    assert G.min() >= 1
    kmax = min(200, int(math.log(20.0 / n) / math.log1p(-p_tot)))   # >= 20 expected in the tail bin
    counts = np.bincount(np.minimum(G, kmax), minlength=kmax + 1)[1:]
    pk = p_tot * (1 - p_tot) ** np.arange(kmax)
    pk[-1] = (1 - p_tot) ** (kmax - 1)
    assert stats.chisquare(counts, n * pk).pvalue > 1e-5
    assert abs(G.mean() * p_tot - 1) < 0.01


def check_two_harmonic_waveform():
    """The electrical-asymmetry drive V0 [cos(wt) + cos(2wt)] (Sec. III): 2 V0 at
    wt = 0, -V0 at wt = pi/2, 0 at wt = pi, and its minimum -9/8 V0 where
    cos(wt) = -1/4."""
    p = W.discharge_small()
    p.update(v0_volt=100.0, v2_volt=100.0, phase_rad=0.0, phase2_rad=0.0, steps_per_cycle=400)
    assert abs(P.voltage(p, 0) - 200.0) < 1e-12
    assert abs(P.voltage(p, 100) + 100.0) < 1e-12
    assert abs(P.voltage(p, 200)) < 1e-12
    assert abs(P.voltage(p, 400) - 200.0) < 1e-12
    vmin = min(P.voltage(p, l) for l in range(400))
    assert abs(vmin + 112.5) < 0.05


def check_circuit_vacuum_divider():
    """Blocking capacitor without space charge: the capacitor C_B and the gap
    C_gap = eps0 / L divide the source, Phi_0(t) = (C_gap V(0) + C_B V(t) + q) /
    (C_gap + C_B) with q the net charge the electrode absorbed; the potential is
    linear across the gap."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=150.0, phase_rad=0.3, p_pa=1.0)
    cb = 2.0e-9
    p.update(cb_f_m2=cb)
    d = P.Discharge(p)
    L = p["gap_m"]
    cg = C.EPS0 / L
    V0 = P.voltage(p, 0)
    Phi = d.field(0)[4]
    assert abs(Phi[0] - V0) < 1e-12 * abs(V0)                 # the capacitor starts uncharged
    assert abs(d.sigma_init - cg * V0) < 1e-9 * abs(cg * V0)
    for l, n_net in ((37, 0), (123, 5000), (250, -20000)):
        d.n_abs_net = n_net
        q = C.E_CHARGE * d.d["w"] * n_net
        Phi = d.field(l)[4]
        want = (cg * V0 + cb * P.voltage(p, l) + q) / (cg + cb)
        assert abs(Phi[0] - want) <= 1e-9 * max(abs(want), 1.0), (l, Phi[0], want)
        x = np.arange(Phi.size) / (Phi.size - 1)
        assert np.allclose(Phi, want * (1 - x), rtol=0, atol=1e-9 * max(abs(want), 1.0))


def check_circuit_large_capacitor_is_the_ideal_source():
    """As C_B grows the electrode follows the source: with space charge present the
    circuit solve tends to the Dirichlet solve Phi_0 = V(t)."""
    p = W.discharge_small(seed=4)
    p.update(cb_f_m2=1.0e3)
    d = P.Discharge(p)
    d.field(0)
    d.run(3)
    d.n_abs_net += 123
    Qe, Qi, rho, V, Phi, E = d.field(d.step_index)
    ref = P.solve_potential(rho, V, d.d["dx"])
    assert np.max(np.abs(Phi - ref)) < 1e-6 * max(np.max(np.abs(ref)), 1.0)


def check_skip_cap_memoryless(p_tot=3e-5, n=200000):
    """A wait longer than WAIT_CAP is cut there and redrawn; the total wait to the
    first real examination keeps the geometric law P(T > k) = (1 - P)^k (the law
    has no memory), with no excess at the cap."""
    ids = np.arange(n, dtype=np.uint64)
    U = R.draw(ids, 0, R.tag(1, R.SKIP), 9, 4)
    nxt, redraw, _ = P.skip(U[:, 0], 0, p_tot, P.WAIT_CAP)
    assert np.all(nxt[redraw] == P.WAIT_CAP) and np.all(nxt[~redraw] <= P.WAIT_CAP)
    for _ in range(60):
        if not redraw.any():
            break
        k = np.nonzero(redraw)[0]
        Uk = R.draw(ids[k], nxt[k], R.tag(1, R.COLL), 9, 4)
        nxt[k], redraw[k], _ = P.skip(Uk[:, 7], nxt[k], p_tot, P.WAIT_CAP)
    assert not redraw.any()
    T = nxt
    assert T.min() >= 1
    # 40 bins of equal geometric probability
    q = np.arange(1, 40) / 40.0
    edges = np.ceil(np.log1p(-q) / math.log1p(-p_tot)).astype(np.int64)
    counts = np.bincount(np.searchsorted(edges, T, side="left"), minlength=40)
    cdf = 1.0 - (1.0 - p_tot) ** np.concatenate([edges, [np.iinfo(np.int64).max // 2]]).astype(np.float64)
    pk = np.diff(np.concatenate([[0.0], np.minimum(cdf, 1.0)]))
    assert stats.chisquare(counts, n * pk / pk.sum()).pvalue > 1e-5
    assert abs(T.mean() * p_tot - 1) < 0.02
    # no pile-up at the cut: P(T in (cap - 50, cap + 50]) as for the geometric law
    near = np.count_nonzero((T > P.WAIT_CAP - 50) & (T <= P.WAIT_CAP + 50))
    expect = n * ((1 - p_tot) ** (P.WAIT_CAP - 50) - (1 - p_tot) ** (P.WAIT_CAP + 50))
    assert abs(near - expect) < 6 * math.sqrt(expect)


def check_redraw_examination_only_redraws(n=20000):
    """At a cut wait's examination step the particle is not collided: no process is
    selected, its velocity is the pushed one, and its next examination comes from
    U7 of that step's candidate draw."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0, p_pa=5.0)
    d = P.Discharge(p, load=False, wait_cap=P.WAIT_CAP)
    N = d.d["N"]
    rng = np.random.default_rng(8)
    v = rng.normal(size=(n, 3)) * 3e5
    _set_state(d, 0, np.full(n, N / 2 + 0.25), v)
    _set_state(d, 1, np.zeros(0), np.zeros((0, 3)))
    d.sp[0].next[:] = 0
    d.sp[0].redraw[:] = True
    rec = d.step(record=True)
    assert d.acc["candidates"][0] == 0 and sum(d.acc["collisions"]) == 0 and d.acc["births"] == 0
    assert "proc_0" not in rec
    sp = d.sp[0]
    assert np.array_equal(sp.v, v)
    U = R.draw(sp.id, 0, R.tag(0, R.COLL), p["seed"], p["case_id"])
    nxt, redraw, _ = P.skip(U[:, 7], 0, d.d["p_tot"][0], P.WAIT_CAP)
    assert np.array_equal(sp.next, nxt) and np.array_equal(sp.redraw, redraw)


def check_elastic_excitation_ionisation_kinematics(n=300000):
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0, p_pa=50.0)
    d = P.Discharge(p, load=False)
    N = d.d["N"]
    m, M, mr = C.M_E, C.M_AR, d.d["mr"][0]
    rng = np.random.default_rng(6)
    eps0 = 40.0
    g = math.sqrt(2 * eps0 * C.E_CHARGE / mr)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    _set_state(d, 0, np.full(n, N / 2 + 0.5), g * dirs)
    _set_state(d, 1, np.zeros(0), np.zeros((0, 3)))
    d.sp[0].next[:] = 0
    v_before = g * dirs
    # the push moves x only (no field), so v^(l+1/2) = v_before
    rec = d.step(record=True)
    proc = rec["proc_0"]
    vafter = d.sp[0].v[:n]            # births are appended after the parents
    Vcm = (m / (m + M)) * v_before
    gprime = np.linalg.norm(vafter - Vcm, axis=1) * (m + M) / M
    el = proc == P.P_EL
    assert np.allclose(gprime[el], g, rtol=1e-12)
    # mean fractional energy loss of isotropic elastic scattering: 2 m M / (m + M)^2
    e_before = 0.5 * m * g ** 2
    e_after = 0.5 * m * np.sum(vafter[el] ** 2, axis=1)
    mean_loss = np.mean(1 - e_after / e_before)
    expect = 2 * m * M / (m + M) ** 2
    assert abs(mean_loss / expect - 1) < 0.02, (mean_loss, expect)
    ex = proc == P.P_EXC
    assert ex.sum() > 1000
    assert np.allclose(0.5 * mr * gprime[ex] ** 2 / C.E_CHARGE, eps0 - 11.5, rtol=1e-9)
    io = proc == P.P_ION
    assert io.sum() > 1000
    e1 = 0.5 * m * np.sum(vafter[io] ** 2, axis=1) / C.E_CHARGE
    assert np.allclose(e1, (eps0 - 15.8) / 2, rtol=1e-9)
    w0, xt_c, v2, _ = rec["birth_e"]
    assert np.allclose(0.5 * m * np.sum(v2 ** 2, axis=1) / C.E_CHARGE, (eps0 - 15.8) / 2, rtol=1e-9)
    assert np.array_equal(xt_c, d.sp[0].xt[:n][io])     # born at the parent x^(l+1)
    # isotropy of the scattered directions
    u = (vafter[el] - Vcm[el]) / np.linalg.norm(vafter[el] - Vcm[el], axis=1)[:, None]
    assert np.all(np.abs(u.mean(axis=0)) < 0.01)
    assert np.all(np.abs((u ** 2).mean(axis=0) - 1 / 3) < 0.01)


def check_charge_exchange_thermalises(n=400000, beam_ev=100.0):
    """After resonant charge exchange the ion carries the thermal partner's
    velocity.  For a fast beam (|v| >> thermal speed) the |v - v_bg| weighting of
    the selection barely biases the partner, so <v'^2> = 3 k_B T / M."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0, p_pa=20.0)
    d = P.Discharge(p, load=False)
    N = d.d["N"]
    rng = np.random.default_rng(8)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    v = math.sqrt(2 * beam_ev * C.E_CHARGE / C.M_AR) * dirs
    _set_state(d, 0, np.zeros(0), np.zeros((0, 3)))
    _set_state(d, 1, np.full(n, N / 2 + 0.5), v)
    d.sp[1].next[:] = 0
    rec = d.step(record=True)
    cx = rec["proc_1"] == P.P_CX
    assert cx.sum() > 100000
    v2 = np.sum(d.sp[1].v[cx] ** 2, axis=1)
    assert abs(v2.mean() / (3 * C.K_B * p["t_gas_k"] / C.M_AR) - 1) < 0.01
    assert np.all(np.abs(d.sp[1].v[cx].mean(axis=0)) < 3.0)


def check_loading_moments(n=200000):
    p = W.discharge(0.025, 64, 100.0, 400, 1.0, n, 1e15, case_id=9)
    d = P.Discharge(p)
    for s, T, m in ((0, p["te_ev"], C.M_E), (1, p["ti_ev"], C.M_AR)):
        v = d.sp[s].v
        assert np.allclose(v.var(axis=0), T * C.E_CHARGE / m, rtol=0.015)
        assert stats.kstest(d.sp[s].xt / 64.0, "uniform").pvalue > 1e-4


def check_density_normalisation():
    """sum_m n_m dx_m = w * (time-averaged number of super-particles), exactly in
    the integer accumulators."""
    p = W.discharge_small()
    d = P.Discharge(p)
    counts = []
    for _ in range(30):
        counts.append(len(d.sp[0]))
        d.step()
    out = d.sample_diagnostics()
    dx = d.d["dx"]
    vol = np.full(d.d["N"] + 1, dx)
    vol[0] = vol[-1] = dx / 2
    assert d.acc["sumQ"][0].sum() == 2 ** 32 * sum(counts)
    assert abs(np.sum(out["ne"] * vol) / (d.d["w"] * np.mean(counts)) - 1) < 1e-12


# ------------------------------------------------- phase-resolved averages, fluxes
def check_flux_over_density_is_the_beam_velocity(n_steps=12):
    """Field-free, collisionless drift of two beams, electrons at +v_e and ions at
    -v_i, from positions bunched unevenly inside the cells: every node's mean
    velocity Gamma / n equals its beam's velocity (the density and the flux are
    sampled at the same positions), and Gamma integrates to w N_p v over the
    gap."""
    p = field_free_case(v0_volt=0.0, flux_profiles=1)
    d = P.Discharge(p, load=False)
    N, dx, dt, w = d.d["N"], d.d["dx"], d.d["dt"], d.d["w"]
    rng = np.random.default_rng(5)
    n = 3000
    # cell index skewed toward the left, offset within the cell clustered at 0.15
    cells = np.floor(N * rng.beta(1.5, 3.0, n)).astype(np.int64)
    xt = cells + np.clip(rng.normal(0.15, 0.05, n), 0.0, 0.999)
    ve, vi = 0.3 * dx / dt, 0.2 * dx / dt          # 0.3 and 0.2 cells per step
    for s, vx in ((0, ve), (1, -vi)):
        v = np.zeros((n, 3))
        v[:, 0] = vx
        _set_state(d, s, xt.copy(), v)
    counts = []
    for _ in range(n_steps):
        counts.append((len(d.sp[0]), len(d.sp[1])))
        d.step()
    out = d.sample_diagnostics()
    vol = np.full(N + 1, dx)
    vol[0] = vol[N] = dx / 2
    for key, dens, vx in (("e", out["ne"], ve), ("i", out["ni"], -vi)):
        held = dens > 1e-3 * dens.max()
        assert np.allclose(out["u_" + key][held], vx, rtol=1e-6, atol=0)
        assert np.all(out["u_" + key][~held & (dens == 0)] == 0)
    for s, key, vx in ((0, "e", ve), (1, "i", -vi)):
        mean_np = np.mean([c[s] for c in counts])
        total = np.sum(out["gamma_" + key] * vol)
        assert abs(total / (w * mean_np * vx) - 1) < 1e-12


def _bin_mean_of_cosine(V0, theta, d, m):
    """(1/m) sum_{k<m} V0 cos(theta + k d), from the closed form of the sum of
    cosines in arithmetic progression."""
    return V0 * math.sin(m * d / 2) / (m * math.sin(d / 2)) * math.cos(theta + (m - 1) * d / 2)


def check_phase_bins_resolve_the_drive(n_phase=8, start=130):
    """Vacuum gap driven by V0 cos(wt + phase): over two whole RF periods each
    phase bin holds 2 N_t / n_phase steps, its potential at the driven electrode
    is the drive averaged over the bin's steps (a closed-form sum), the potential
    is linear across the gap, and the bins weighted by their step counts give the
    window's time averages."""
    Nt = 400
    p = field_free_case(v0_volt=100.0, phase_rad=0.7, steps_per_cycle=Nt, n_phase=n_phase,
                        np_e=40, np_i=40, capacity_e=40, capacity_i=40)
    d = P.Discharge(p)
    for _ in range(start):
        d.step()
    d.reset_diagnostics()
    for _ in range(2 * Nt):
        d.step()
    tot = d.sample_diagnostics()
    m = Nt // n_phase
    dth = 2 * math.pi / Nt
    N = d.d["N"]
    acc = {k: np.zeros(N + 1) for k in ("ne", "ni", "phi")}
    for b in range(n_phase):
        o = d.sample_phase(b)
        assert o["n_steps"] == 2 * m
        want = _bin_mean_of_cosine(p["v0_volt"], 2 * math.pi * b * m / Nt + p["phase_rad"], dth, m)
        assert abs(o["phi"][0] - want) <= 1e-9 * p["v0_volt"], (b, o["phi"][0], want)
        assert np.allclose(o["phi"], o["phi"][0] * (1 - np.arange(N + 1) / N), rtol=0, atol=1e-9)
        for k in acc:
            acc[k] += o[k] * o["n_steps"]
    scale = {"ne": np.max(tot["ne"]), "ni": np.max(tot["ni"]), "phi": p["v0_volt"]}
    for k in acc:
        assert np.allclose(acc[k] / (2 * Nt), tot[k], rtol=0, atol=1e-12 * scale[k]), k


# ------------------------------------------------------------ joint energy-angle
def check_iead_of_a_known_beam():
    """Ions sent into the field-free target at known energies and angles land in
    the joint energy-angle bins their (E, theta) name (4 eV by 1 degree), and the
    joint histogram's marginals are the 1 eV and 0.25 degree histograms grouped."""
    p = field_free_case(v0_volt=0.0)
    d = P.Discharge(p, load=False)
    dx, dt = d.d["dx"], d.d["dt"]
    E = np.array([10.3, 10.3, 57.9, 121.0, 121.0, 250.2, 250.2, 250.2])
    th = np.array([0.1, 3.7, 0.6, 12.4, 12.6, 44.0, 0.9, 80.2])
    speed = np.sqrt(2 * E * C.E_CHARGE / C.M_AR)
    v = np.stack([-speed * np.cos(np.radians(th)), speed * np.sin(np.radians(th)), np.zeros(E.size)], axis=1)
    xt = -v[:, 0] * dt / dx * 0.5                   # each crosses x = 0 within the step
    _set_state(d, 1, xt, v)
    _set_state(d, 0, np.array([32.0]), np.zeros((1, 3)))
    d.step()
    h = d.acc["iead"][0]
    want = np.zeros_like(h)
    for e, t in zip(E, th):
        want[int(e) // 4, int(t / 0.25) // 4] += 1
    assert np.array_equal(h, want)
    assert not d.acc["iead"][1].any()
    nb = d.d["n_ebins"]
    pad = np.zeros(-(-nb // 4) * 4 - nb, dtype=np.int64)
    for el in (0, 1):
        e_marg = np.concatenate([d.acc["iedf"][el], pad]).reshape(-1, 4).sum(axis=1)
        a_marg = d.acc["iadf"][el].reshape(-1, 4).sum(axis=1)
        assert np.array_equal(d.acc["iead"][el].sum(axis=1), e_marg)
        assert np.array_equal(d.acc["iead"][el].sum(axis=0), a_marg)


# ------------------------------------------------------------ charge exchange rate
def mean_relative_speed(v0, s):
    """<|v0 - V|> for V Maxwellian with per-component spread s (a beam of speed v0
    through a thermal gas): the relative speed g has the density
    g / (v0 s sqrt(2 pi)) [exp(-(g - v0)^2 / (2 s^2)) - exp(-(g + v0)^2 / (2 s^2))],
    integrated numerically and checked against the closed form
    s sqrt(2/pi) exp(-l^2/2) + (v0 + s^2/v0) erf(l/sqrt 2), l = v0 / s."""
    from scipy import integrate, special
    f = lambda g: g * g / (v0 * s * math.sqrt(2 * math.pi)) * (
        math.exp(-(g - v0) ** 2 / (2 * s * s)) - math.exp(-(g + v0) ** 2 / (2 * s * s)))
    hi = v0 + 12 * s
    num = integrate.quad(f, 0.0, hi, limit=200, epsabs=0, epsrel=1e-12)[0]
    lam = v0 / s
    closed = s * math.sqrt(2 / math.pi) * math.exp(-lam * lam / 2) + (v0 + s * s / v0) * special.erf(lam / math.sqrt(2))
    assert abs(num / closed - 1) < 1e-9, (num, closed)
    return num


def _ion_beam_candidates(beam_ev, n, seed=9):
    """Field-free Ar+ at one speed in random directions, every ion a candidate
    of step 0; returns the discharge after that step and its record."""
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0, p_pa=20.0)
    d = P.Discharge(p, load=False)
    N = d.d["N"]
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    v0 = math.sqrt(2 * beam_ev * C.E_CHARGE / C.M_AR)
    _set_state(d, 0, np.zeros(0), np.zeros((0, 3)))
    _set_state(d, 1, np.full(n, N / 2 + 0.5), v0 * dirs)
    d.sp[1].next[:] = 0
    rec = d.step(record=True)
    return p, d, rec, v0


def check_charge_exchange_rate(n=400000):
    """Given a candidate, an Ar+ of speed v0 charge-exchanges with probability
    n sigma_cx g / nu_max for the drawn partner's relative speed g (the selection
    rule after Eq. (6)): over many candidates the fraction is
    n sigma_cx <g> / nu_max, with <g> the mean relative speed of a beam through the
    Maxwellian gas.  Checked at a thermal beam (0.05 eV, where the partner's
    motion sets most of g) and a fast one (100 eV)."""
    for beam_ev in (0.05, 100.0):
        p, d, rec, v0 = _ion_beam_candidates(beam_ev, n)
        s = math.sqrt(C.K_B * p["t_gas_k"] / C.M_AR)
        frac = d.d["n_gas"] * p["sigma_cx"] * mean_relative_speed(v0, s) / d.d["nu_max"][1]
        k = int(np.count_nonzero(rec["proc_1"] == P.P_CX))
        lo, hi = stats.binom.interval(1 - 1e-6, n, frac)
        assert lo <= k <= hi, (beam_ev, k, n * frac)
        assert d.acc["candidates"][1] == n and d.acc["collisions"][4] == k


def check_ion_majorant_bounds_the_capped_energy(n=200000):
    """The ions' majorant of Eq. (6) is n sigma_cx g_cap with g_cap the speed at
    the energy cap plus ten thermal widths of the partner: no candidate at the
    cap exceeds it, while a beam 21 % above the cap in energy (10 % in speed, far
    more than ten thermal widths here) does, in a fraction set by the partner's
    Gaussian spread along the beam."""
    from scipy import special
    p = field_free_case(flags=P.NO_SELF_FIELD, v0_volt=0.0, p_pa=20.0)
    cap = p["ecap_i_ev"]
    _, d, _, _ = _ion_beam_candidates(cap, n)
    assert d.acc["overflow"][1] == 0
    _, d, _, v0 = _ion_beam_candidates(1.21 * cap, n)
    s = math.sqrt(C.K_B * p["t_gas_k"] / C.M_AR)
    g_cap = math.sqrt(2 * cap * C.E_CHARGE / C.M_AR) + 10 * s
    # |v0 - V| > g_cap; with g_cap << v0 and s << v0 this is the partner's
    # component against the beam exceeding g_cap - v0 (< 0): nearly every candidate
    p_over = 0.5 * special.erfc((g_cap - v0) / (s * math.sqrt(2)))
    k = int(d.acc["overflow"][1])
    lo, hi = stats.binom.interval(1 - 1e-6, n, min(p_over, 1 - 1e-12))
    assert lo - 50 <= k <= hi, (k, n * p_over)


# ------------------------------------------------------- wall flux and impact energy
def check_wall_flux_and_impact_energy(n_steps=400):
    """Uniform beams in a field-free, collisionless gap, one per species and
    electrode: N_b particles of energy E on an even lattice over the 2 d next to
    the electrode they drift into, d = v n dt the distance the beam drifts in the
    window of n steps.  Half of each lattice arrives, so each (species,
    electrode) receives its beam's particle flux n_b v with n_b = w N_b / (2 d)
    the density a super-particle weight w gives, i.e. w N_b / (2 n dt); the ions
    arrive at normal incidence with 1/2 M v^2, each in its 1 eV bin."""
    p = field_free_case(v0_volt=0.0)
    d = P.Discharge(p, load=False)
    N, dx, dt, w, L = d.d["N"], d.d["dx"], d.d["dt"], d.d["w"], p["gap_m"]
    beams = {(1, 0): (20000, 50.5), (1, 1): (8000, 20.5), (0, 0): (12000, 0.05), (0, 1): (16000, 0.03)}
    for s in (0, 1):
        xs, vs = [], []
        for el in (0, 1):
            n_b, E = beams[(s, el)]
            v = math.sqrt(2 * E * C.E_CHARGE / (C.M_AR if s else C.M_E))
            lat = (np.arange(n_b) + 0.5) / n_b * 2 * v * n_steps * dt      # distance from the electrode
            x = lat if el == 0 else L - lat
            assert x.min() > 0 and x.max() < L
            vv = np.zeros((n_b, 3))
            vv[:, 0] = -v if el == 0 else v
            xs.append(x / dx)
            vs.append(vv)
        _set_state(d, s, np.concatenate(xs), np.concatenate(vs))
    for _ in range(n_steps):
        d.step()
    out = d.sample_diagnostics()
    assert out["avg_steps"] == n_steps
    for (s, el), (n_b, E) in beams.items():
        assert out["absorbed"][s][el] == n_b // 2, (s, el, out["absorbed"])
        want = w * n_b / (2 * n_steps * dt)
        assert abs(out["flux"][s][el] / want - 1) < 1e-12, (s, el, out["flux"][s][el], want)
        if s == 1:
            assert abs(out["mean_ion_energy"][el] / E - 1) < 1e-12, (el, out["mean_ion_energy"])
            assert out["iedf"][el][int(E)] == n_b // 2 and out["iedf"][el].sum() == n_b // 2
            assert out["iadf"][el][0] == n_b // 2
