"""Brute-force Monte Carlo of the continuum gain term of eq. C22_general.

Test infrastructure.  Written from the definition only (no oracle code):
G(p1) = 1/(2 E1 g) int dPi_2 dPi_3 dPi_4 (2pi)^4 delta^4(p1+p2-p3-p4) |M|^2 f3 f4.
The (p3, p4) integral is done in the centre-of-mass frame of p1+p2, where it
is p*/(16 pi^2 sqrt(s)) int dOmega*, and the outgoing momenta are boosted to
the lab.  p2 is sampled log-uniformly in momentum and uniformly in the cosine
of its angle to p1; the CM direction uniformly on the sphere.
"""
import numpy as np


def gain(p1, f, mass=1.0, gdof=1.0, m2=1.0, lo=1e-3, hi=30.0, ns=2_000_000, seed=1):
    """Gain term (dilute) at momentum p1: (mean, standard error)."""
    g, l = collision(p1, f, 0, mass, gdof, m2, lo, hi, ns, seed)
    return g


def collision(p1, f, eta, mass=1.0, gdof=1.0, m2=1.0, lo=1e-3, hi=30.0, ns=2_000_000, seed=1):
    """Gain and loss parts of eq. C22_general with the statistical factor of
    eq. Lambda_quantum: gain = f3 f4 (1 + eta f1)(1 + eta f2), loss = f1 f2
    (1 + eta f3)(1 + eta f4).  Returns ((gain, se), (loss, se))."""
    rng = np.random.default_rng(seed)
    e1 = np.sqrt(p1 * p1 + mass * mass)
    p2 = np.exp(rng.uniform(np.log(lo), np.log(hi), ns))
    c2 = rng.uniform(-1.0, 1.0, ns)
    s2 = np.sqrt(1.0 - c2 * c2)
    e2 = np.sqrt(p2 * p2 + mass * mass)
    P = np.stack([p2 * s2, np.zeros(ns), p1 + p2 * c2], 1)
    P0 = e1 + e2
    s = P0 * P0 - (P * P).sum(1)
    rs = np.sqrt(s)
    pstar = np.sqrt(np.maximum(s / 4.0 - mass * mass, 0.0))
    ct = rng.uniform(-1.0, 1.0, ns)
    ph = rng.uniform(0.0, 2.0 * np.pi, ns)
    st = np.sqrt(1.0 - ct * ct)
    nhat = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1)
    beta = P / P0[:, None]
    b2 = (beta * beta).sum(1)
    gam = 1.0 / np.sqrt(1.0 - b2)

    def boost(pv, e):
        bp = (beta * pv).sum(1)
        coef = (gam - 1.0) * bp / b2 + gam * e
        return pv + coef[:, None] * beta

    e3 = rs / 2.0
    p3 = boost(pstar[:, None] * nhat, e3)
    p4 = boost(-pstar[:, None] * nhat, e3)
    q3 = np.sqrt((p3 * p3).sum(1))
    q4 = np.sqrt((p4 * p4).sum(1))
    vol = (np.log(hi) - np.log(lo)) * 2.0 * 4.0 * np.pi
    meas = (2.0 * np.pi * p2 ** 3 / ((2.0 * np.pi) ** 3 * 2.0 * e2)) \
        * (pstar / (16.0 * np.pi ** 2 * rs)) * m2 * vol / (2.0 * e1 * gdof)
    f1, f2, f3, f4 = f(np.array([p1]))[0], f(p2), f(q3), f(q4)
    g = meas * f3 * f4 * (1.0 + eta * f1) * (1.0 + eta * f2)
    l = meas * f1 * f2 * (1.0 + eta * f3) * (1.0 + eta * f4)
    se = lambda v: float(v.std() / np.sqrt(ns))
    return (float(g.mean()), se(g)), (float(l.mean()), se(l))
