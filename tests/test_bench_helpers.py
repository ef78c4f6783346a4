"""Host checks of the growth-rate fits used by the physics workloads (synthetic signals)."""
import math

import numpy as np

import bench


def _signal(rate, floor=0.01, amp0=1e-4, cap=50.0, dt=0.04, tmax=80.0):
    t = np.arange(0.0, tmax, dt)
    return t, np.minimum(floor + amp0 * np.exp(2.0 * rate * t), cap)


def test_max_growth_recovers_the_rate_of_an_exponential_over_a_noise_floor():
    for rate in (0.08, 0.2, 0.35):
        t, w = _signal(rate)
        r, (a, b) = bench.max_growth(t, w, 6.0)
        assert abs(r / rate - 1.0) < 0.01, (rate, r)
        assert b - a <= 6.0 + 1e-9 and w[np.searchsorted(t, b)] <= w.max()


def test_max_growth_without_growth_is_nan():
    t = np.arange(0.0, 20.0, 0.04)
    r, _ = bench.max_growth(t, np.full_like(t, 0.5), 4.0)
    assert math.isnan(r)


def test_growth_rate_fit_on_the_linear_phase():
    t, w = _signal(0.3, floor=1e-6, amp0=1e-9, cap=1.0)
    best, whole, (t0, t1) = bench.growth_rate_fit(t, w)
    assert abs(best / 0.3 - 1.0) < 0.01 and abs(whole / 0.3 - 1.0) < 0.05 and t0 < t1


def test_two_stream_rate_matches_the_cold_dispersion_relation():
    # the unstable root must satisfy 1 = a [1/(w - kv)^2 + 1/(w + kv)^2] with w = i gamma
    k, v0 = 2.9452, 0.2
    g = bench.two_stream_rate(k, v0)
    a = 0.5 * (1 - v0 * v0) ** 1.5
    w = 1j * g
    assert abs(a * (1 / (w - k * v0) ** 2 + 1 / (w + k * v0) ** 2) - 1.0) < 1e-12
    assert abs(g - 0.342867) < 1e-6


def test_lds_model_bound_from_its_instruction_counts():
    # cubic weights: 300 64-bit atomics at 6.3 clk and 192 paired reads at 4 clk per 64
    # particles, 256 CUs at 2.4 GHz
    clk = (300 * 6.3 + 192 * 4.0) / 64.0
    assert bench.lds_bound_updates_per_s(3) == 256 * 2.4e9 / clk
    # quadratic weights: 3 * 3 * 4 * 4 atomics and 6 * 27 / 2 paired reads
    clk2 = (144 * 6.3 + 81 * 4.0) / 64.0
    assert bench.lds_bound_updates_per_s(2) == 256 * 2.4e9 / clk2


def test_measured_traffic_is_used_only_for_the_kernel_sources_it_was_taken_on(monkeypatch):
    import os
    vals = {}
    for line in open(os.path.join(bench.ROOT, "profiles", "k_gpd32_pair_mj_256_counters.md")):
        line = line.strip()
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k] = v
    n = int(vals["particles"])
    per_byte_f = float(vals["copy_fetch_kib"]) * 1024.0 / float(vals["copy_bytes"])
    per_byte_w = float(vals["copy_write_kib"]) * 1024.0 / float(vals["copy_bytes"])
    want = (float(vals["fetch_kib_per_launch"]) * 1024.0 / per_byte_f
            + float(vals["write_kib_per_launch"]) * 1024.0 / per_byte_w)
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: vals["kernel_source_digest"])
    assert bench.measured_traffic(n) == want
    assert 1.0 < want / (56.0 * n) < 10.0  # against the algorithmic 56 B per particle
    assert bench.measured_traffic(n + 1) is None  # another workload
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
    assert bench.measured_traffic(n) is None  # counters taken on other kernel sources
