"""Host logic of the energy meter (no GPU needed): missing sources are
reported as None with a note, RAPL counters are differenced with their wrap
range, and power samples are integrated by the trapezoid rule."""
import os

from paper_2509_19294_amd import energy


def test_meter_without_gpu_reports_none(monkeypatch):
    monkeypatch.setattr(energy, "_amdsmi", lambda: (None, "amdsmi not importable: test"))
    monkeypatch.setattr(energy, "_rapl_files", lambda: [])
    with energy.EnergyMeter() as em:
        pass
    r = em.result()
    assert r["gpu_energy_j"] is None and r["host_energy_j"] is None
    assert r["gpu_power_samples"] == 0 and r["gpu_energy_from_power_samples_j"] is None
    assert any("amdsmi" in n for n in r["notes"]) and any("RAPL" in n for n in r["notes"])
    assert r["wall_s"] is not None and r["wall_s"] >= 0


def test_rapl_difference_with_wrap(tmp_path, monkeypatch):
    monkeypatch.setattr(energy, "_amdsmi", lambda: (None, "no"))
    pkgs = []
    for k, (start, rng) in enumerate(((1_000_000, 10_000_000), (9_500_000, 10_000_000))):
        d = tmp_path / f"pkg{k}"
        d.mkdir()
        (d / "energy_uj").write_text(f"{start}\n")
        (d / "max_energy_range_uj").write_text(f"{rng}\n")
        pkgs.append((str(d / "energy_uj"), str(d / "max_energy_range_uj")))
    monkeypatch.setattr(energy, "_rapl_files", lambda: pkgs)
    em = energy.EnergyMeter()
    em.__enter__()
    # package 0 advances by 2 J, package 1 wraps and advances by 1 J
    open(pkgs[0][0], "w").write("3000000\n")
    open(pkgs[1][0], "w").write("500000\n")
    em.__exit__(None, None, None)
    assert abs(em.result()["host_energy_j"] - 3.0) < 1e-9


def test_power_samples_trapezoid():
    em = energy.EnergyMeter()
    em._t0, em._t1 = 0.0, 2.0
    em._samples = [(0.0, 100.0), (1.0, 300.0), (2.0, 300.0)]
    r = em.result()
    assert r["gpu_energy_from_power_samples_j"] == 500.0
    assert r["gpu_peak_power_w"] == 300.0 and r["gpu_power_samples"] == 3


def test_counter_that_did_not_advance_is_none():
    em = energy.EnergyMeter()
    em._t0, em._t1 = 0.0, 0.2
    em._e0 = em._e1 = 1234.5
    r = em.result()
    assert r["gpu_energy_j"] is None and r["gpu_mean_power_w"] is None
    assert any("did not advance" in n for n in r["notes"])

