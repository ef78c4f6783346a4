"""Host checks of the growth-rate fits used by the physics workloads (synthetic signals)."""
import math

import numpy as np
import pytest

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


def test_roofline_fractions_from_a_counter_summary(monkeypatch):
    # one launch of 1.2e9 particles in 100 ms: 56 B each against 8 TB/s; 2.4e10 counted VALU
    # wavefront instructions against one per clock per CU; 3.0e9 ds_add against the probe rate
    n, ms = 1_200_000_000, 100.0
    cs = {"kernel_source_digest": "x", "particles": n, "valu_insts_per_launch": 2.4e10,
          "lds_insts_per_launch": 5.0e9, "lds_atomic_insts_per_launch": 3.0e9}
    monkeypatch.setattr(bench, "read_counter_summary", lambda p: cs if p == n else None)
    monkeypatch.setattr(bench, "measured_traffic", lambda p: None)
    r = bench.kernel_roofline(n, ms)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["frac"] - n * 56 / 0.1 / 8e12) < 1e-4
    assert abs(r["valu"]["frac"] - 2.4e10 / 0.1 / (256 * 2.4e9)) < 1e-4
    assert abs(r["lds_atomic"]["frac"] - 3.0e9 / 0.1 / (256 * 2.4e9 / bench.LDS_CLK_PER_WAVE_ATOMIC)) < 1e-4
    assert r["valu"]["insts_per_64_particles"] == round(2.4e10 * 64 / n, 1)
    assert r["binding"] == max(("hbm", r["frac"]), ("valu", r["valu"]["frac"]),
                               ("lds", r["lds_atomic"]["frac"]), key=lambda t: t[1])[0]
    # with the LDS-active counter the LDS pipe's busy fraction decides for the LDS
    cs.update(lds_active_per_launch=0.9 * 8e8 / 8 * 256, gui_active_per_launch=8e8)
    r = bench.kernel_roofline(n, ms)
    assert abs(r["lds_atomic"]["lds_pipe_busy"] - 0.9) < 1e-9 and r["binding"] == "lds"
    # no summary for these sources: only the HBM figure
    r = bench.kernel_roofline(n + 1, ms)
    assert r["valu"] is None and r["lds_atomic"] is None and r["frac"] > 0


def test_counter_summary_round_trip(tmp_path, monkeypatch):
    # a rocprofv3-style CSV of two passes (three launches of the particle kernel and one copy)
    # gives a summary whose machine-read lines reproduce the per-launch means
    import csv
    k = "void pp::k_gpd32<3, pp::TileCT<3, 4, 4, 4, false> >(pp::Gpd32Args)"
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    passes = {"a": {"SQ_INSTS_VALU": [9e9, 1e10, 1.2e10], "GRBM_GUI_ACTIVE": [8e8, 8e8, 8e8]},
              "b": {"FETCH_SIZE": [5e7, 6e7, 8e7]}}
    for name, cnt in passes.items():
        d = tmp_path / name
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=cols)
            w.writeheader()
            for i in range(3):
                for c, v in cnt.items():
                    w.writerow(dict(Dispatch_Id=10 + i, Kernel_Name=k, Counter_Name=c, Counter_Value=v[i],
                                    Start_Timestamp=0, End_Timestamp=int(100e6)))
            w.writerow(dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name=list(cnt)[0],
                            Counter_Value=2.0e6, Start_Timestamp=0, End_Timestamp=1000))
    out = tmp_path / "summary.md"
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "d" * 16)
    bench.counter_summary([str(tmp_path / "a"), str(tmp_path / "b")], str(out), 1_000_000, ["cmd a", "cmd b"])
    text = out.read_text()
    monkeypatch.setattr(bench, "os", bench.os)
    vals = dict(line[2:].split(": ", 1) for line in text.splitlines() if line.startswith("- "))
    assert float(vals["valu_insts_per_launch"]) == 1.1e10  # launches after the first
    assert float(vals["fetch_kib_per_launch"]) == 7e7
    assert float(vals["kernel_ms"]) == 100.0
    assert vals["kernel_source_digest"] == "d" * 16 and "cmd a" in text


def test_counter_summary_sums_the_split_elementwise_pass(tmp_path, monkeypatch):
    # the elementwise calibration pass over 4 GiB comes as several dispatches (torch splits a
    # tensor this large): their counters and durations are summed, so the factors per byte and
    # the stream rate refer to the whole 4 GiB; the fastest plain stream becomes the roofline's
    # stream reference
    import csv
    k = "void pp::k_gpd32<3, pp::TileCT<3, 4, 4, 4, false> >(pp::Gpd32Args)"
    ew = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>"
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    gib4_kib = 4 * (1 << 30) / 1024.0
    d = tmp_path / "p"
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i in range(2):  # two launches of the particle kernel, 80 ms each
            w.writerow(dict(Dispatch_Id=10 + i, Kernel_Name=k, Counter_Name="FETCH_SIZE", Counter_Value=4e7,
                            Start_Timestamp=0, End_Timestamp=int(80e6)))
        # the copy: 2 ms, counter half the bytes read
        w.writerow(dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name="FETCH_SIZE",
                        Counter_Value=0.5 * gib4_kib, Start_Timestamp=0, End_Timestamp=int(2e6)))
        # the elementwise pass: two dispatches of 0.7 ms, each reading 2 GiB (counter: half of it)
        for i in range(2):
            w.writerow(dict(Dispatch_Id=2 + i, Kernel_Name=ew, Counter_Name="FETCH_SIZE",
                            Counter_Value=0.25 * gib4_kib, Start_Timestamp=0, End_Timestamp=int(0.7e6)))
    out = tmp_path / "summary.md"
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "e" * 16)
    bench.counter_summary([str(d)], str(out), 1_000_000, ["cmd"])
    text = out.read_text()
    vals = dict(line[2:].split(": ", 1) for line in text.splitlines() if line.startswith("- "))
    assert float(vals["ew_fetch_kib"]) == pytest.approx(0.5 * gib4_kib)  # both dispatches
    assert float(vals["ew_gbs"]) == pytest.approx(8 * (1 << 30) / 1.4e-3 / 1e9)  # 8 GiB in 1.4 ms
    assert float(vals["copy_gbs"]) == pytest.approx(8 * (1 << 30) / 2e-3 / 1e9)
    assert "2 dispatches" in text and "(factor 0.500)" in text
    # the roofline takes the faster stream as its reference
    cs = {k: float(v) for k, v in vals.items() if k != "kernel_source_digest"}
    monkeypatch.setattr(bench, "read_counter_summary", lambda n: cs)
    monkeypatch.setattr(bench, "measured_traffic", lambda n: None)
    r = bench.kernel_roofline(1_000_000_000, 80.0)  # 700 GB/s algorithmic
    assert r["stream_peak_gbs"] == pytest.approx(cs["ew_gbs"], abs=0.05)  # reported to 0.1 GB/s
    assert r["frac_of_stream"] == pytest.approx(r["achieved"] / cs["ew_gbs"], rel=1e-3)


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


def test_mode_rates_finds_the_growing_bins():
    # three bins grow at 0.2, 0.15 and 0.1 from t = 10 on over a flat floor and stop at 50
    # (saturation); the others stay at the floor; a +-k pair appears once; the linear phase
    # ends at t = 55
    import math

    import numpy as np
    tb = np.arange(0, 70.01, 0.5)
    kv = np.array([0, 1, 2, -2, -1])
    W = np.full((len(tb), 5, 5, 5), 1e-6)
    grow = np.exp(2 * np.clip(tb - 10.0, 0.0, 40.0))
    W[:, 1, 2, 0] *= grow ** 0.2  # kz = 1, ky = 2, kx = 0
    W[:, 4, 3, 0] *= grow ** 0.2  # its mirror -k
    W[:, 2, 0, 1] *= grow ** 0.15
    W[:, 0, 1, 1] *= grow ** 0.1
    dk = 2 * math.pi / 12.8
    m = bench.mode_rates(tb, kv, W, dk, 55.0, top=5)
    assert len(m) == 3  # the floor bins never leave their noise
    assert [round(x["rate"], 9) for x in m] == [0.2, 0.15, 0.1]
    assert np.allclose(m[0]["k"], [0.0, 2 * dk, dk]) or np.allclose(m[0]["k"], [0.0, -2 * dk, -dk])
    assert abs(m[0]["angle_deg"] - math.degrees(math.atan2(2, 1))) < 1e-9
    assert abs(m[2]["abs_k"] - math.sqrt(2) * dk) < 1e-12
    # a linear phase ending before the bins leave their floor leaves nothing to fit
    assert bench.mode_rates(tb, kv, W, dk, 12.0) == []
