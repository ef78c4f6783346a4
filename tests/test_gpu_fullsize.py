"""GPU parity at the full sizes of the benchmark workloads, built on the device and stepped
as the benchmark times them: the 256^3 pair plasma (32 particles per cell per species,
1,073,741,824 particles), the 128x32x32 two-stream box (two beams of 32 per cell on a quiet
lattice over an ion background, cell 0.1) and the 1024x512x1 Kelvin-Helmholtz layer (64 per
cell per species, flat 8x8x1 tiles), each in the split FP32 and the plain FP64 form.

The oracle cannot step these in seconds, so a seeded sample of particles is followed
through one step and compared with the oracle's steps 1-3 for those particles on the same
fields (the bar of the small parity cases: u within 1e-5 relative and positions within
1e-6 cell for FP32, 1e-12 for FP64); the rest is checked through properties that hold at
any size: discrete charge conservation of the deposited current and Gauss's law after the
field step (normalised residuals <= 1e-6 for FP32, 1e-10 for FP64), no flagged particle,
and every particle present exactly once."""
import sys

import numpy as np
import pytest

from _state import periodic_diff, rel_inf, rel_l2
from paper_1211_4575_amd import inputs as I

pytestmark = pytest.mark.gpu

SAMPLE = 4096


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair_mj(bench, pp, ind, torch, split):
    n, ppc = (256, 256, 256), 32
    run, npart = bench.make_pair_mj_run(pp, ind, torch, n, ppc, 1.0, split, with_id=True)
    return run, npart, ((-1.0, 1.0, 1.0 / ppc), (1.0, 1.0, 1.0 / ppc)), dict(n=n, dt=0.4)


def _arrays(torch, npart, split, nsp=2):
    dev = torch.device("cuda:0")
    rt = torch.float32 if split else torch.float64
    cells = [torch.empty(npart, dtype=torch.int32, device=dev) for _ in range(nsp)] if split else None
    offs = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(nsp)]
    us = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(nsp)]
    return cells, offs, us


def _species(split, cells, offs, us, qmw):
    out = []
    for s, (q, m, w) in enumerate(qmw):
        sp = dict(q=q, m=m, w=w, u=us[s])
        sp.update(dict(cell=cells[s], off=offs[s]) if split else dict(pos=offs[s]))
        out.append(sp)
    return out


def _two_stream(bench, pp, ind, torch, split):
    n, per_dim, dx = (128, 32, 32), (4, 4, 2), 0.1
    ppc = per_dim[0] * per_dim[1] * per_dim[2]
    npart = n[0] * n[1] * n[2] * ppc
    cells, offs, us = _arrays(torch, npart, split)
    ind.two_stream_lattice(bench.SEED, 2, n, per_dim, 0.2, 0.01, ind.split_mode(split, 3), cells,
                           [[o[d] for d in range(3)] for o in offs], [[u[d] for d in range(3)] for u in us],
                           torch.cuda.current_stream().cuda_stream)
    qmw = ((-1.0, 1.0, 0.5 / ppc), (-1.0, 1.0, 0.5 / ppc))
    P = pp.make_params(n, d=(dx, dx, dx), dt=0.4 * dx, shape_order=3, field_order=6, alpha=0.55,
                       precision=pp.PP_PREC_FP32_SPLIT if split else pp.PP_PREC_FP64,
                       relax_tol=1e-8 if split else 1e-14, relax_max_iter=100, rho_background=1.0)
    run = pp.Run(P, _species(split, cells, offs, us, qmw), with_id=True)
    return run, npart, qmw, dict(n=n, d=(dx, dx, dx), dt=0.4 * dx)


def _kelvin_helmholtz(bench, pp, ind, torch, split):
    n, ppc = (1024, 512, 1), 64
    npart = n[0] * n[1] * n[2] * ppc
    cells, offs, us = _arrays(torch, npart, split)
    ind.kelvin_helmholtz(bench.SEED, n, 0, npart, 0.2, 8.0, 0.02, ind.split_mode(split, 3), cells,
                         [[o[d] for d in range(3)] for o in offs], [[u[d] for d in range(3)] for u in us],
                         torch.cuda.current_stream().cuda_stream)
    qmw = ((-1.0, 1.0, 1.0 / ppc), (1.0, 25.0, 1.0 / ppc))
    P = pp.make_params(n, shape_order=3, field_order=6, dt=0.4, alpha=0.55,
                       precision=pp.PP_PREC_FP32_SPLIT if split else pp.PP_PREC_FP64,
                       relax_tol=1e-8 if split else 1e-14, relax_max_iter=100)
    run = pp.Run(P, _species(split, cells, offs, us, qmw), with_id=True)
    return run, npart, qmw, dict(n=n, dt=0.4)


WORKLOADS = {"pair_mj_256": _pair_mj, "two_stream_128x32x32": _two_stream, "kh_1024x512x1": _kelvin_helmholtz}


def _sample(run, torch, s, ids):
    """Positions (float64, cell units) and momenta (host arrays) of the particles with the
    given ids, and how many ids of the species occur exactly once."""
    T = run.particle_tensors(s)
    n = T["id"].shape[0]
    slot = torch.empty(n, dtype=torch.int64, device=T["id"].device)
    slot[T["id"]] = torch.arange(n, dtype=torch.int64, device=slot.device)
    q = slot[torch.as_tensor(ids, device=slot.device)]
    pos = np.stack([T["pos"][d][q].cpu().numpy() for d in range(3)])
    out = dict(pos=pos, u=np.stack([T["u"][d][q].cpu().numpy() for d in range(3)]))
    if T["cell"] is not None:
        out["cell"] = T["cell"][q].cpu().numpy()
    present = int(torch.count_nonzero(torch.bincount(T["id"], minlength=n) == 1))
    del slot, q, T
    return out, present


@pytest.mark.parametrize("split", [True, False], ids=["fp32_split", "fp64"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_full_size_step_sampled_against_oracle(orc, name, split):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import bench
    from paper_1211_4575_amd import inputs_device as ind
    from paper_1211_4575_amd import pp

    form = "fp32_split" if split else "fp64"
    _say("full size: loading", name, form)
    run, npart, qmw, okw = WORKLOADS[name](bench, pp, ind, torch, split)
    n = okw["n"]
    try:
        run.step()  # the fields are non-zero from here on
        _say("full size: sampling before the step", name, form)
        E = run.E.cpu().numpy()
        B = run.B.cpu().numpy()
        rng = np.random.default_rng(4575)
        ids = [np.sort(rng.choice(npart, SAMPLE, replace=False)) for _ in qmw]
        before = [_sample(run, torch, s, ids[s])[0] for s in range(len(qmw))]
        run.diagnostics(pp.PP_DIAG_RHO)  # the charge density before the step, for continuity
        run.step()
        _say("full size: sampling after the step", name, form)
        after = []
        for s in range(len(qmw)):
            a, present = _sample(run, torch, s, ids[s])
            assert present == npart, (s, present)
            after.append(a)
        d = run.diagnostics(pp.PP_DIAG_ALL)
        assert d.flags == 0
        bar = 1e-6 if split else 1e-10
        assert d.cc_max / d.rho_ref <= bar, d.cc_max / d.rho_ref
        assert d.gauss_max / d.rho_ref <= bar, d.gauss_max / d.rho_ref
    finally:
        run.close()
        del run
        torch.cuda.empty_cache()

    P = orc.make_params(shape_order=3, field_order=6, alpha=0.55, **okw)
    J = np.zeros_like(E)
    tol_x, tol_u = (1e-6, 1e-5) if split else (1e-12, 1e-12)
    for s, (q, m, w) in enumerate(qmw):
        b, a = before[s], after[s]
        pos = np.ascontiguousarray(I.from_split(b["cell"], b["pos"], n) if split else b["pos"].astype(np.float64))
        u = np.ascontiguousarray(b["u"].astype(np.float64))
        orc.step_species(P, q, m, w, pos, u, E, B, J)
        X = I.from_split(a["cell"], a["pos"], n) if split else a["pos"]
        assert np.max(np.abs(periodic_diff(X, pos, n))) < tol_x, s
        assert rel_inf(a["u"].astype(np.float64), u) < tol_u, s
        if split:
            assert np.all(a["pos"] >= 0.0) and np.all(a["pos"] < 2.0)
        assert np.max(np.abs(a["u"] - b["u"])) > 0.0  # the sample did feel the fields


def test_full_size_field_step_current_and_residual_against_oracle(orc):
    """The benchmark's 256^3 split FP32 step, element by element where the oracle can follow
    it: (1) the field step as the benchmark runs it (tiled kernels, relax_tol 1e-8 at most 100
    sweeps) from the GPU's E^n, B^n and J^{n+1}, against the oracle's field step from the same
    three arrays (the OpenMP build, bitwise the plain one for this step; relaxed to 1e-10):
    E^{n+1} and B^{n+1} within 1e-5 (L2, relative to the change); (2) the measured relaxation
    residual max |rhs - A B| / max |rhs| at or below 1e-8; (3) the current on an 8^3 window:
    the GPU's field-order current J_O turned back into the second-order one with the banded
    stencil of eqs. "jj6d"/"penta" (J_2 = T J_O along each component's axis, T = (c, b+c,
    a+b+c, b+c, c)) against the oracle's second-order current of every particle within reach
    of the window, within 1e-5 (L2, relative)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import bench
    from paper_1211_4575_amd import inputs_device as ind
    from paper_1211_4575_amd import pp

    _say("full size field step: loading")
    run, npart, qmw, okw = _pair_mj(bench, pp, ind, torch, True)
    n = okw["n"]
    w0, W, reach = (100, 37, 211), 8, 4
    try:
        run.step()  # non-zero fields from here on
        E0 = run.E.cpu().numpy()
        B0 = run.B.cpu().numpy()
        # the particles whose cell lies within `reach` cells of the window (periodic)
        near = []
        for s in range(len(qmw)):
            T = run.particle_tensors(s)
            c = T["cell"].to(torch.int64)
            ijk = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
            m = torch.ones_like(c, dtype=torch.bool)
            for d in range(3):
                rel = (ijk[d] - (w0[d] - reach)) % n[d]
                m &= rel < W + 2 * reach
            q = torch.nonzero(m).flatten()
            near.append(dict(cell=T["cell"][q].cpu().numpy(), pos=np.stack([T["pos"][d][q].cpu().numpy() for d in range(3)]),
                             u=np.stack([T["u"][d][q].cpu().numpy() for d in range(3)])))
            del T, c, m, q, ijk
        _say("full size field step: particles near the window", [x["cell"].size for x in near])
        run.gather_push_deposit()
        J = run.J.cpu().numpy()
        run.sort()
        run.field_step()
        E1 = run.E.cpu().numpy()
        B1 = run.B.cpu().numpy()
        d = run.diagnostics(pp.PP_DIAG_RELAX)
        _say("full size field step: measured residual", d.relax_resid_meas, "sweeps", d.relax_iters)
        assert d.relax_resid_meas <= 1e-8, d.relax_resid_meas
        assert d.flags == 0
    finally:
        run.close()
        del run
        torch.cuda.empty_cache()

    P = orc.make_params(shape_order=3, field_order=6, alpha=0.55, relax_tol=1e-10, relax_max_iter=200, **okw)
    Eo, Bo = E0.copy(), B0.copy()
    with orc.openmp():
        _say("full size field step: oracle field step on", orc.num_threads(), "threads")
        it, res = orc.field_step(P, Eo, Bo, J)
    _say("full size field step: oracle sweeps", it, "residual", res)
    errE, errB = rel_l2(E1 - E0, Eo - E0), rel_l2(B1 - B0, Bo - B0)
    _say("full size field step: dE", errE, "dB", errB)
    assert errE < 1e-5 and errB < 1e-5

    # the window's second-order current from the oracle
    Jo = np.zeros_like(E0)
    for s, (q, m, w) in enumerate(qmw):
        x = near[s]
        pos = np.ascontiguousarray(I.from_split(x["cell"], x["pos"], n))
        u = np.ascontiguousarray(x["u"].astype(np.float64))
        assert orc.step_species(P, q, m, w, pos, u, E0, B0, Jo) == 0
    a = orc.fd_coeffs(6)
    taps = {0: a[0] + a[1] + a[2], 1: a[1] + a[2], 2: a[2]}
    sl = [np.arange(w0[d], w0[d] + W) % n[d] for d in range(3)]
    got, want = [], []
    for comp in range(3):
        T2 = np.zeros((W, W, W))
        for o in range(-2, 3):
            idx = list(sl)
            idx[comp] = (sl[comp] + o) % n[comp]
            T2 += taps[abs(o)] * J[comp][np.ix_(idx[2], idx[1], idx[0])]
        got.append(T2)
        want.append(Jo[comp][np.ix_(sl[2], sl[1], sl[0])])
    errJ = rel_l2(np.array(got), np.array(want))
    _say("full size current window: J_2 error", errJ)
    assert errJ < 1e-5
