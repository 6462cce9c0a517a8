"""Pins of the drift oracle (oracle/drift.py; Fig. 2's drifting, spreading clouds).

The widths are checked against simulated random walks of electrons (a Brownian path's
variance after time t is 2 D t per axis), the attenuation against simulated exponential
lifetimes, the projection against points built on a wire's line, the time against the
drift of whole ticks; plus the handling of depositions that are not drifted and the
plane-major row layout.
"""
import numpy as np

from oracle import drift as OD

RNG = np.random.default_rng(11)


def params(**kw):
    base = dict(drift_speed=0.16, diffusion_l=4.0e-6, diffusion_t=8.8e-6, lifetime=8000.0, tick=0.5,
                angles=(np.radians(60.0), np.radians(-60.0), 0.0), pitches=(0.3, 0.3, 0.3),
                wire_offsets=(1200.0, 1200.0, 1728.0), time_offsets=(0.0, 2.0, 4.0))
    base.update(kw)
    return OD.DriftParams(**base)


def one(x, y=10.0, z=20.0, t0=5.0, q=1e4, sl0=0.05, st0=0.03, prm=None):
    prm = prm or params()
    return OD.drift_rows([x], [y], [z], [t0], [q], [sl0], [st0], [3], [77], prm)


def random_walk_spread(D, t, sigma0, n=20000, steps=200):
    """Sample variance of electron positions along one axis after a random walk of time t."""
    pos = RNG.normal(0.0, sigma0, n)
    dt = t / steps
    for _ in range(steps):
        pos += RNG.normal(0.0, np.sqrt(2.0 * D * dt), n)
    return pos.var(ddof=1)


def test_widths_follow_random_walks():
    prm = params()
    x = 150.0  # cm: about 940 us of drift
    r = one(x, prm=prm)
    td = x / prm.drift_speed
    n = 20000
    vt = random_walk_spread(prm.diffusion_t, td, 0.03, n)
    vl = random_walk_spread(prm.diffusion_l, td, 0.05, n)
    # transverse width across the plane's wires (pitches) and longitudinal width in ticks
    sp = r["sigma_p"][0] * prm.pitches[0]
    stt = r["sigma_t"][0] * prm.drift_speed * prm.tick
    tol = 5.0 * np.sqrt(2.0 / (n - 1))
    assert abs(vt / sp ** 2 - 1.0) < tol
    assert abs(vl / stt ** 2 - 1.0) < tol
    # longer drifts spread more, and the width at x = 0 is the initial one
    assert one(200.0)["sigma_p"][0] > r["sigma_p"][0]
    r0 = one(0.0)
    assert np.isclose(r0["sigma_p"][0] * 0.3, 0.03, rtol=1e-14)
    assert np.isclose(r0["sigma_t"][0] * prm.drift_speed * prm.tick, 0.05, rtol=1e-14)


def test_attenuation_follows_exponential_lifetimes():
    prm = params(lifetime=3000.0)
    x = 200.0
    td = x / prm.drift_speed
    n = 200000
    survive = np.mean(RNG.exponential(prm.lifetime, n) > td)
    frac = one(x, q=1.0, prm=prm)["q"][0]
    assert abs(survive - frac) < 5.0 * np.sqrt(frac * (1 - frac) / n)
    # no attenuation without a lifetime, none at x = 0
    assert one(x, prm=params(lifetime=0.0))["q"][0] == 1e4
    assert one(0.0)["q"][0] == 1e4


def test_projection_on_wire_lines():
    prm = params()
    for k, (th, P, off) in enumerate(zip(prm.angles, prm.pitches, prm.wire_offsets)):
        wires = RNG.integers(0, 2400, 200).astype(np.float64)
        s = RNG.uniform(-300, 300, 200)
        # wire w's line: its points at signed distance (w - off) P from the origin along the
        # normal (sin th, cos th) in (y, z), shifted along the wire direction (cos th, -sin th)
        d = (wires - off) * P
        y = d * np.sin(th) + s * np.cos(th)
        z = d * np.cos(th) - s * np.sin(th)
        n = wires.size
        r = OD.drift_rows(np.full(n, 10.0), y, z, np.zeros(n), np.ones(n), np.zeros(n), np.zeros(n),
                          np.zeros(n), np.arange(n), prm)
        sel = r["plane"] == k
        assert np.allclose(r["p"][sel], wires, rtol=0, atol=1e-9)
    # the collection plane (theta = 0) reads z, a plane at 90 degrees reads y
    r = one(5.0, y=3.3, z=7.5, prm=params(angles=(0.0, np.pi / 2, 0.0)))
    assert np.isclose(r["p"][0], 7.5 / 0.3 + 1200.0) and np.isclose(r["p"][1], 3.3 / 0.3 + 1200.0)


def test_time_is_drift_plus_offsets_in_ticks():
    prm = params()
    r0 = one(0.0, t0=7.0)
    assert np.allclose(r0["t"], (7.0 + np.array(prm.time_offsets)) / prm.tick, rtol=1e-15)
    m = 1234
    r = one(m * prm.drift_speed * prm.tick, t0=7.0)
    assert np.allclose(r["t"] - r0["t"], m, rtol=0, atol=1e-9)


def test_depositions_not_drifted_carry_no_charge():
    prm = params()
    x = np.array([-1.0, np.nan, 10.0, 10.0, 10.0])
    y = np.array([1.0, 1.0, np.inf, 1.0, 1.0])
    q = np.array([5e3, 5e3, 5e3, 5e3, np.nan])
    n = x.size
    r = OD.drift_rows(x, y, np.ones(n), np.zeros(n), q, np.zeros(n), np.zeros(n), np.zeros(n), np.arange(n), prm)
    qq = r["q"].reshape(3, n)
    assert np.all(qq[:, [0, 1, 2, 4]] == 0) and np.all(qq[:, 3] > 0)


def test_rows_are_plane_major():
    prm = params()
    n = 7
    r = OD.drift_rows(np.linspace(1, 100, n), np.ones(n), np.ones(n), np.zeros(n), np.ones(n), np.zeros(n),
                      np.zeros(n), np.arange(n) % 2, np.arange(10, 10 + n), prm)
    assert r["plane"].tolist() == [0] * n + [1] * n + [2] * n
    assert r["depo_id"].tolist() == list(range(10, 10 + n)) * 3
    assert r["event"].tolist() == (np.arange(n) % 2).tolist() * 3
