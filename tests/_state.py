"""Seeded synthetic states for parity tests (no method arithmetic here except the curl used
to make a divergence-free B, which goes through the oracle)."""
import numpy as np


def random_state(orc, n, ppc, seed, uth=0.3, e_amp=0.05, b_amp=0.3, nspecies=2, pair=True, d=(1.0, 1.0, 1.0)):
    """Random particles in an n-cell box and random fields with div B = 0.
    Returns (species list of dicts with q, m, w, pos, u; E; B)."""
    rng = np.random.default_rng(seed)
    ncell = n[0] * n[1] * n[2]
    npart = ncell * ppc
    pos0 = rng.uniform(0, 1, (3, npart)) * np.array(n, dtype=np.float64)[:, None]
    pos0 = np.where(pos0 >= np.array(n)[:, None], 0.0, pos0)
    species = []
    charges = [-1.0, 1.0, -1.0, 1.0]
    masses = [1.0, 1.0, 4.0, 25.0]
    for s in range(nspecies):
        if pair or s == 0:
            pos = pos0.copy()
        else:
            pos = rng.uniform(0, 1, (3, npart)) * np.array(n, dtype=np.float64)[:, None]
            pos = np.where(pos >= np.array(n)[:, None], 0.0, pos)
        u = rng.normal(0.0, uth, (3, npart))
        species.append(dict(q=charges[s], m=masses[s], w=1.0 / ppc, pos=np.ascontiguousarray(pos),
                            u=np.ascontiguousarray(u)))
    shape = (3, n[2], n[1], n[0])
    E = e_amp * rng.normal(size=shape)
    P = orc.make_params(n=n, d=d)
    B = b_amp * orc.curl_up(P, rng.normal(size=shape)) / 2.0
    return species, np.ascontiguousarray(E), np.ascontiguousarray(B)


def periodic_diff(a, b, n):
    d = a - b
    n = np.asarray(n, dtype=np.float64)[:, None]
    return d - n * np.round(d / n)


def rel_inf(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def rel_l2(a, b):
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def poisson_E(orc, P, rho):
    """E = (up derivatives of phi) with div_down E = rho - mean(rho): the potential solves the
    field-order discrete Poisson equation by FFT, with the exact symbol of the composed
    down(up) stencils taken from the oracle's derivatives of a unit impulse."""
    shape = rho.shape
    sym = np.zeros(shape)
    delta = np.zeros(shape)
    delta[0, 0, 0] = 1.0
    for d in range(3):
        sym += np.fft.fftn(orc.deriv(P, orc.deriv(P, delta, d, True), d, False)).real
    rh = np.fft.fftn(rho)
    rh[0, 0, 0] = 0.0
    sym[0, 0, 0] = 1.0
    phi = np.ascontiguousarray(np.fft.ifftn(rh / sym).real)
    return np.stack([orc.deriv(P, phi, d, True) for d in range(3)])
