"""Shared helpers of the GPU parity tests: move a state between the GPU case
(internal units: cells, cells per step) and the oracle (cells, m/s)."""
import numpy as np

from oracle import pic as P

F32_EPS = 2.0 ** -23


def oracle_from_gpu(case, p):
    """An oracle discharge holding exactly the GPU case's current state, on the
    GPU's examination schedule (waits cut at WAIT_CAP)."""
    d = P.Discharge(p, load=False, wait_cap=P.WAIT_CAP)
    info = case.info()
    vs = info["dx"] / info["dt"]
    for s in (0, 1):
        g = case.get_particles(s)
        sp = d.sp[s]
        sp.xt = g["xt"].astype(np.float64)
        sp.v = np.stack([g["ux"], g["uy"], g["uz"]], axis=1) * vs
        sp.id = g["id"].astype(np.uint64)
        sp.next, sp.redraw = split_next(g["next"])
    d.step_index = case.sample_diagnostics()["step"]
    if p.get("cb_f_m2", 0.0) > 0.0:
        f = case.get_fields()
        d.sigma_init, d.n_abs_net = f["sigma_init"], int(f["n_absorbed_net"])
    return d


def split_next(code):
    """The interface's next-examination code -> (step, redraw flag): bit 31 marks an
    examination that only redraws the wait; all bits set means never."""
    code = np.asarray(code).astype(np.int64)
    never = code == P.NEVER
    step = np.where(never, P.NEVER, code & 0x7FFFFFFF)
    return step, ~never & ((code >> 31) & 1).astype(bool)


def next_code(step, redraw):
    """Inverse of split_next."""
    step = np.asarray(step, dtype=np.int64)
    return np.where(step == P.NEVER, P.NEVER, step | (np.asarray(redraw, dtype=np.int64) << 31))


def by_id(ids, *arrays):
    o = np.argsort(ids, kind="stable")
    return (ids[o],) + tuple(a[o] for a in arrays)


def gpu_state_si(case, s):
    g = case.get_particles(s)
    info = case.info()
    vs = info["dx"] / info["dt"]
    v = np.stack([g["ux"], g["uy"], g["uz"]], axis=1) * vs
    return by_id(g["id"], g["xt"], v, g["next"].astype(np.int64))


def oracle_state(d, s):
    sp = d.sp[s]
    return by_id(sp.id, sp.xt, sp.v, next_code(sp.next, sp.redraw))


def snapshot(case):
    """Particles of both species in id order, the grid state and the diagnostics."""
    out = []
    for s in (0, 1):
        g = case.get_particles(s)
        o = np.argsort(g["id"])
        out.append({k: v[o] for k, v in g.items()})
    f = case.get_fields()
    d = case.sample_diagnostics()
    return out, f, d


def assert_same(a, b):
    """Two snapshots agree bit for bit."""
    for s in (0, 1):
        for k in a[0][s]:
            assert np.array_equal(a[0][s][k], b[0][s][k]), (s, k)
    for k in ("qe", "qi", "E", "phi"):
        assert np.array_equal(a[1][k], b[1][k]), k
    for k in ("ne", "ni", "phi", "iedf", "iadf", "absorbed", "collisions", "candidates"):
        assert np.array_equal(a[2][k], b[2][k]), k
