"""Linear theory and seeded eigenmode of the relativistic beam-plasma system of the mixed-mode
test (Sec. VIII.C): a cold neutral beam (electrons and ions, density n_b, Lorentz factor G
along z) through a cold neutral background at rest (density n_p), c = eps0 = 1, total
electron plasma frequency 1.

Theory (test infrastructure, independent of the method's code): the cold relativistic
two-fluid equations linearised about the uniform drifting state, with Maxwell's equations, for
one Fourier mode exp(i(k.x - w t)):

    w dn_s = (k.v_s) dn_s + n_s k.dv_s,          dv_s = (du_s - v_s (v_s.du_s)) / g_s
    w du_s = (k.v_s) du_s + i (q_s/m_s)(dE + v_s x dB)
    w dB   = k x dE
    w dE   = -k x dB - i sum_s q_s (n_s dv_s + dn_s v_s)

an eigenvalue problem w x = M x whose largest imaginary eigenvalue is the growth rate at k.
The particles of the particle-in-cell method feel the field through their B-spline weights and
deposit through them as well, which multiplies the coupling by the squared form factor
S(k)^2, S = prod_d sinc(k_d dx / 2)^(O+1) for weights of order O (finite-size particle theory),
taken into account by scaling every charge by S.
"""
import math

import numpy as np

GAMMA_B = 4.0
MASS_ION = 1836.0


def _cross(a):
    return np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])


def populations(gamma_b=GAMMA_B, n_b=0.1, n_p=0.9, mass_ion=MASS_ION):
    """(q, m, n, v_z) of beam electrons, beam ions, background electrons, background ions."""
    v = math.sqrt(1.0 - 1.0 / gamma_b ** 2)
    return [(-1.0, 1.0, n_b, v), (1.0, mass_ion, n_b, v), (-1.0, 1.0, n_p, 0.0), (1.0, mass_ion, n_p, 0.0)]


def operator(k, pops, charge_scale=1.0):
    """The matrix M of w x = M x; x = (dn, du[3]) per population, then dE[3], dB[3]."""
    k = np.asarray(k, dtype=float)
    ns = len(pops)
    M = np.zeros((4 * ns + 6, 4 * ns + 6), dtype=complex)
    iE, iB = 4 * ns, 4 * ns + 3
    for s, (q, m, n0, vz) in enumerate(pops):
        q = q * charge_scale
        v0 = np.array([0.0, 0.0, vz])
        g0 = 1.0 / math.sqrt(1.0 - vz * vz)
        D = (np.eye(3) - np.outer(v0, v0)) / g0
        kv = float(k @ v0)
        b = 4 * s
        M[b, b] = kv
        M[b, b + 1:b + 4] = n0 * (k @ D)
        M[b + 1:b + 4, b + 1:b + 4] = kv * np.eye(3)
        M[b + 1:b + 4, iE:iE + 3] = 1j * q / m * np.eye(3)
        M[b + 1:b + 4, iB:iB + 3] = 1j * q / m * _cross(v0)
        M[iE:iE + 3, b + 1:b + 4] += -1j * q * n0 * D
        M[iE:iE + 3, b] += -1j * q * v0
    M[iB:iB + 3, iE:iE + 3] = _cross(k)
    M[iE:iE + 3, iB:iB + 3] = -_cross(k)
    return M


def form_factor(k, dx, order):
    return float(np.prod([np.sinc(k[d] * dx / (2 * np.pi)) ** (order + 1) for d in range(3)]))


def growing_mode(k, pops, charge_scale=1.0):
    """(w, eigenvector) of the fastest-growing mode at k."""
    w, vecs = np.linalg.eig(operator(k, pops, charge_scale))
    j = int(np.argmax(w.imag))
    return w[j], vecs[:, j]


def seeded_state(n, dx, per_dim=(1, 1, 2), amp=1e-3, order=3):
    """The fastest-growing mode at the box's fundamental wave vector (2 pi / L_x, 0, 2 pi / L_z)
    seeded on a quiet lattice: every population on the same lattice of per_dim particles per
    cell, displaced by the mode's Lagrangian displacement xi_s = i dv_s / (w - k.v_s) and given
    its momentum perturbation du_s (beam-electron |du| = amp); E and B set to the mode's fields
    at their staggered positions.  Returns (species dicts, E, B, k, growth rate with the form
    factor, growth rate of the fluid theory)."""
    pops = populations()
    L = np.array(n, dtype=float) * dx
    k = np.array([2 * math.pi / L[0], 0.0, 2 * math.pi / L[2]])
    S = form_factor(k, dx, order)
    w, x = growing_mode(k, pops, charge_scale=S)
    w_fluid, _ = growing_mode(k, pops)
    x = x / np.max(np.abs(x[1:4])) * amp
    ppc = per_dim[0] * per_dim[1] * per_dim[2]
    grids = np.meshgrid(*[np.arange(n[d] * per_dim[d]) for d in range(3)], indexing="ij")
    X0 = np.stack([(grids[d].ravel() + 0.5) / per_dim[d] for d in range(3)])  # cell units
    ph = np.exp(1j * (k @ (X0 * dx)))
    species = []
    for s, (q, m, n0, vz) in enumerate(pops):
        v0 = np.array([0.0, 0.0, vz])
        g0 = 1.0 / math.sqrt(1.0 - vz * vz)
        du = x[4 * s + 1:4 * s + 4]
        dv = (np.eye(3) - np.outer(v0, v0)) @ du / g0
        xi = 1j * dv / (w - k @ v0)
        pos = np.mod(X0 + np.real(np.outer(xi, ph)) / dx, np.array(n, dtype=float)[:, None])
        pos = np.where(pos >= np.array(n)[:, None], 0.0, pos)
        u = np.zeros_like(pos)
        u[2] = g0 * vz
        u += np.real(np.outer(du, ph))
        species.append(dict(q=q, m=m, w=n0 / ppc, pos=np.ascontiguousarray(pos), u=np.ascontiguousarray(u)))

    def on(shift):
        i, j, kk = np.meshgrid(*[np.arange(n[d]) + shift[d] for d in range(3)], indexing="ij")
        return np.exp(1j * dx * (k[0] * i + k[1] * j + k[2] * kk)).transpose(2, 1, 0)  # [z, y, x]

    dE, dB = x[16:19], x[19:22]
    E = np.stack([np.real(dE[c] * on([0.5 if d == c else 0.0 for d in range(3)])) for c in range(3)])
    B = np.stack([np.real(dB[c] * on([0.0 if d == c else 0.5 for d in range(3)])) for c in range(3)])
    return species, np.ascontiguousarray(E), np.ascontiguousarray(B), k, float(w.imag), float(w_fluid.imag)


def energy_rate(t, W):
    """Growth rate of the field amplitude: half the least-squares log slope of the energy."""
    return 0.5 * float(np.polyfit(np.asarray(t), np.log(np.asarray(W)), 1)[0])
