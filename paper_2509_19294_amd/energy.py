"""Energy-to-solution of a region of host code: GPU energy from the device's
own energy accumulator, GPU power sampled in a background thread, host CPU
package energy from the Linux powercap (RAPL) files when they are readable.

The paper integrates card power sampled at about 1 Hz and reads CPU package
energy through RAPL over the simulation's wall-clock span (Section 4). Here
the GPU's cumulative energy counter gives the integral directly (no sampling
error); the power samples (default 10 Hz) give the mean and the peak. Every
source that is missing or not permitted is reported as None with a note,
never guessed.

    with EnergyMeter() as em:
        run()
    print(em.result())
"""
from __future__ import annotations

import glob
import os
import threading
import time


def _amdsmi():
    try:
        import amdsmi
    except Exception as e:  # pragma: no cover - depends on the machine
        return None, f"amdsmi not importable: {e}"
    return amdsmi, None


def _torch_bus_id(device_index: int):
    """PCI bus number of a torch device, or None."""
    try:
        import torch

        props = torch.cuda.get_device_properties(device_index)
        bus = getattr(props, "pci_bus_id", None)
        return int(bus) if bus is not None else None
    except Exception:
        return None


def _rapl_files():
    """Top-level package energy files of the powercap interface."""
    out = []
    for d in sorted(glob.glob("/sys/class/powercap/*rapl*:[0-9]")):
        f = os.path.join(d, "energy_uj")
        m = os.path.join(d, "max_energy_range_uj")
        if os.path.exists(f):
            out.append((f, m))
    return out


def _read_int(path):
    with open(path) as fh:
        return int(fh.read().strip())


def _open_handle(device_index: int):
    """(amdsmi module, processor handle, notes) for a torch device; the
    handle is None (with a note) when it cannot be found."""
    notes = []
    smi, err = _amdsmi()
    if smi is None:
        return None, None, [err]
    try:
        smi.amdsmi_init()
    except Exception as e:
        return None, None, [f"amdsmi_init failed: {e}"]
    try:
        handles = smi.amdsmi_get_processor_handles()
    except Exception as e:
        return smi, None, [f"no GPU handles: {e}"]
    bus = _torch_bus_id(device_index)
    chosen = None
    if bus is not None:
        for h in handles:
            try:
                bdf = smi.amdsmi_get_gpu_device_bdf(h)  # "dddd:bb:dd.f"
                if int(bdf.split(":")[1], 16) == bus:
                    chosen = h
                    break
            except Exception:
                continue
    if chosen is None and len(handles) == 1:
        chosen = handles[0]
    if chosen is None:
        notes.append(f"could not match torch device {device_index} (bus {bus}) among {len(handles)} GPUs")
    return smi, chosen, notes


def temperatures(device_index: int = 0) -> dict:
    """Edge and hotspot temperatures (degrees C) of a torch device from the
    system-management library; None for a reading it cannot give."""
    out = {"temp_edge_c": None, "temp_hotspot_c": None}
    smi, handle, notes = _open_handle(device_index)
    if smi is None:
        return out
    try:
        if handle is not None:
            types = smi.AmdSmiTemperatureType
            metric = smi.AmdSmiTemperatureMetric.CURRENT
            for key, name in (("temp_edge_c", "EDGE"), ("temp_hotspot_c", "HOTSPOT")):
                try:
                    out[key] = float(smi.amdsmi_get_temp_metric(handle, getattr(types, name), metric))
                except Exception:
                    pass
    finally:
        try:
            smi.amdsmi_shut_down()
        except Exception:
            pass
    return out


def _number(v):
    """A positive reading as float, or None ("N/A" strings, zeros, sentinels)."""
    return float(v) if isinstance(v, (int, float)) and 0 < v < 65535 else None


def gfx_clock_mhz(smi, handle):
    """The graphics clock in MHz: the mean over the XCDs' current clocks
    from the GPU metrics table, else the clock query's current value; None
    when neither can be read."""
    try:
        m = smi.amdsmi_get_gpu_metrics_info(handle)
        per_xcd = [x for x in (_number(v) for v in (m.get("current_gfxclks") or [])) if x]
        if per_xcd:
            return sum(per_xcd) / len(per_xcd)
        v = _number(m.get("current_gfxclk"))
        if v:
            return v
    except Exception:
        pass
    try:
        return _number(smi.amdsmi_get_clock_info(handle, smi.AmdSmiClkType.GFX).get("clk"))
    except Exception:
        return None


class ClockSampler:
    """Context manager sampling the GPU's graphics clock in a background
    thread over its body (default every 50 ms), for stating a throughput
    against the peak at the clock the GPU actually ran at."""

    def __init__(self, device_index: int = 0, interval_s: float = 0.05):
        self.device_index = device_index
        self.interval_s = interval_s
        self.notes: list[str] = []
        self.samples: list[float] = []
        self._smi = self._handle = self._thread = None
        self._stop = threading.Event()

    def _run(self):
        while not self._stop.is_set():
            v = gfx_clock_mhz(self._smi, self._handle)
            if v is not None:
                self.samples.append(v)
            self._stop.wait(self.interval_s)

    def __enter__(self):
        self._smi, self._handle, notes = _open_handle(self.device_index)
        self.notes.extend(notes)
        if self._handle is not None:
            self._thread = threading.Thread(target=self._run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass
        return False

    def result(self) -> dict:
        """Median, min and max of the samples (MHz), None without samples."""
        xs = sorted(self.samples)
        if not xs:
            if not self.notes:
                self.notes.append("no clock sample over the region")
            return {"gfx_mhz_median": None, "gfx_mhz_min": None, "gfx_mhz_max": None,
                    "samples": 0, "notes": self.notes}
        k = len(xs)
        med = xs[k // 2] if k % 2 else 0.5 * (xs[k // 2 - 1] + xs[k // 2])
        return {"gfx_mhz_median": round(med, 1), "gfx_mhz_min": round(xs[0], 1),
                "gfx_mhz_max": round(xs[-1], 1), "samples": k, "notes": self.notes}


class EnergyMeter:
    """Context manager measuring GPU and host energy over its body."""

    def __init__(self, device_index: int = 0, interval_s: float = 0.1):
        self.device_index = device_index
        self.interval_s = interval_s
        self.notes: list[str] = []
        self._smi = None
        self._handle = None
        self._samples: list[tuple[float, float]] = []
        self._stop = threading.Event()
        self._thread = None
        self._e0 = self._e1 = None
        self._rapl0 = self._rapl1 = None
        self._t0 = self._t1 = None

    # -- GPU ------------------------------------------------------------------
    def _open_gpu(self):
        self._smi, self._handle, notes = _open_handle(self.device_index)
        self.notes.extend(notes)

    def _energy_j(self):
        if self._handle is None:
            return None
        try:
            r = self._smi.amdsmi_get_energy_count(self._handle)
            return float(r["energy_accumulator"]) * float(r["counter_resolution"]) * 1e-6
        except Exception as e:
            self.notes.append(f"energy counter unreadable: {e}")
            return None

    def _power_w(self):
        try:
            info = self._smi.amdsmi_get_power_info(self._handle)
        except Exception:
            return None
        for key in ("current_socket_power", "average_socket_power", "socket_power"):
            v = info.get(key)
            if isinstance(v, (int, float)) and v > 0:
                return float(v)
        return None

    def _sampler(self):
        while not self._stop.is_set():
            p = self._power_w()
            if p is not None:
                self._samples.append((time.perf_counter(), p))
            self._stop.wait(self.interval_s)

    # -- host -----------------------------------------------------------------
    def _rapl(self):
        files = _rapl_files()
        if not files:
            return None
        vals = []
        for f, m in files:
            try:
                vals.append((_read_int(f), _read_int(m) if os.path.exists(m) else None))
            except (PermissionError, OSError):
                return None
        return vals

    # -- context --------------------------------------------------------------
    def __enter__(self):
        self._open_gpu()
        self._rapl0 = self._rapl()
        if self._rapl0 is None:
            self.notes.append("host RAPL energy not readable (no powercap files or no permission)")
        self._e0 = self._energy_j()
        if self._handle is not None:
            self._thread = threading.Thread(target=self._sampler, daemon=True)
            self._thread.start()
        self._t0 = time.perf_counter()
        return self

    def __exit__(self, *exc):
        self._t1 = time.perf_counter()
        self._e1 = self._energy_j()
        self._rapl1 = self._rapl() if self._rapl0 is not None else None
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass
        return False

    def result(self) -> dict:
        wall = (self._t1 - self._t0) if self._t1 is not None else None
        gpu_j = None
        if self._e0 is not None and self._e1 is not None:
            gpu_j = self._e1 - self._e0
            if gpu_j <= 0.0:
                # the accumulator advances at the firmware's own interval
                gpu_j = None
                if "energy counter did not advance over the region" not in self.notes:
                    self.notes.append("energy counter did not advance over the region")
        host_j = None
        if self._rapl0 is not None and self._rapl1 is not None:
            host_j = 0.0
            for (a, rng), (b, _) in zip(self._rapl0, self._rapl1):
                d = b - a
                if d < 0 and rng:
                    d += rng
                host_j += d * 1e-6
        powers = [p for _, p in self._samples]
        integ = None
        if len(self._samples) >= 2:
            integ = 0.0
            for (ta, pa), (tb, pb) in zip(self._samples, self._samples[1:]):
                integ += 0.5 * (pa + pb) * (tb - ta)
        return {
            "wall_s": None if wall is None else round(wall, 3),
            "gpu_energy_j": None if gpu_j is None else round(gpu_j, 2),
            "gpu_mean_power_w": None if (gpu_j is None or not wall) else round(gpu_j / wall, 1),
            "gpu_power_samples": len(powers),
            "gpu_peak_power_w": round(max(powers), 1) if powers else None,
            # the paper's method: the trapezoid integral of the power samples
            "gpu_energy_from_power_samples_j": None if integ is None else round(integ, 2),
            "host_energy_j": None if host_j is None else round(host_j, 2),
            "notes": self.notes,
        }
