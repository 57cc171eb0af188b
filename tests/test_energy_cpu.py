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



def test_clock_sampler_without_gpu_reports_none(monkeypatch):
    monkeypatch.setattr(energy, "_amdsmi", lambda: (None, "amdsmi not importable: test"))
    with energy.ClockSampler(interval_s=0.01) as cs:
        pass
    r = cs.result()
    assert r["gfx_mhz_median"] is None and r["samples"] == 0 and r["notes"]


def test_clock_reading_prefers_the_per_xcd_clocks():
    class Smi:
        class AmdSmiClkType:
            GFX = 0

        def __init__(self, metrics, clk):
            self.metrics, self.clk = metrics, clk

        def amdsmi_get_gpu_metrics_info(self, h):
            if self.metrics is None:
                raise RuntimeError("no metrics table")
            return self.metrics

        def amdsmi_get_clock_info(self, h, t):
            return {"clk": self.clk}

    # invalid entries ("N/A", the 0xffff sentinel, 0) are left out of the mean
    per_xcd = {"current_gfxclks": [2400, 2380, "N/A", 65535, 0, 2390, 2410, 2420], "current_gfxclk": 2000}
    assert abs(energy.gfx_clock_mhz(Smi(per_xcd, 1500), None) - 2400.0) < 1e-9
    assert energy.gfx_clock_mhz(Smi({"current_gfxclks": [], "current_gfxclk": 2100}, 1500), None) == 2100.0
    assert energy.gfx_clock_mhz(Smi(None, 1500), None) == 1500.0
    assert energy.gfx_clock_mhz(Smi(None, "N/A"), None) is None


def test_clock_sampler_statistics():
    cs = energy.ClockSampler()
    cs.samples = [2400.0, 2100.0, 2380.0, 2390.0]
    r = cs.result()
    assert r["gfx_mhz_median"] == 2385.0 and r["gfx_mhz_min"] == 2100.0 and r["gfx_mhz_max"] == 2400.0
    assert r["samples"] == 4
