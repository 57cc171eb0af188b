"""Instruction-rate microbenchmarks on gfx950 (the pair kernel's budget).

    python -m paper_2509_19294_amd.microbench [--no-build]

Builds ``libnbody_micro.so`` from ``csrc/microbench.hip`` with the main
library's compiler flags and prints one JSON object. For each case: the
median duration and the issue rate in lane-instructions per compute unit per
clock at the 2.4 GHz peak clock (64 would be one instruction per lane per
clock on all four SIMDs of a CU), and for the synthetic pair loop the
interaction rate with no memory traffic at all (the kernel's ceiling).
"""
from __future__ import annotations

import ctypes
import json
import os
import subprocess

from paper_2509_19294_amd import build as nbuild

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libnbody_micro.so")
SRC = os.path.join(HERE, "csrc", "microbench.hip")

# op -> (name, instructions per chain-iteration)
OPS = {
    0: ("fma_f32", 1),
    1: ("mul_f32", 1),
    2: ("add_f32", 1),
    3: ("rsq_f32", 1),
    4: ("fma_f32_literal", 1),
    5: ("add_f64", 1),
    6: ("fma_f64", 1),
    7: ("add_f64+cvt_f32_f64+add_f32", 3),
    8: ("add_f64+add_f32", 2),
    9: ("13fma_f32+rsq_f32", 14),
    10: ("pair_arith", 14),
    11: ("lds_bcast+4fma_f32", 5),
    12: ("sym_rot_pair_arith", 16 * 19),   # per chain-iteration: 16 pair evaluations
    13: ("pair_arith_mfma_accum", 11),     # 8 VALU + rsq + 2 MFMA per interaction
    # operand placement (inline asm, 16 chains, fixed registers; ilp is 16)
    14: ("fmac_vgpr_three_banks", 1),
    15: ("fmac_vgpr_one_bank", 1),
    16: ("fmac_sgpr_every_instr", 1),
    17: ("fmac_sgpr_one_in_four", 1),
    18: ("sub_sgpr_every_instr", 1),
    19: ("rsq_one_in_nine_fmac", 18 / 16),
    20: ("pair_arith_asm_banked", 56 / 16),   # 4 pairs (14 VALU each) per iteration
}

# (op, ilp, blocks, threads)
CASES = [
    (0, 4, 4096, 256), (0, 8, 4096, 256), (0, 16, 4096, 256),
    (0, 8, 256, 256), (0, 8, 512, 256), (0, 16, 256, 256), (0, 8, 1024, 1024),
    (1, 8, 4096, 256), (2, 8, 4096, 256), (3, 8, 4096, 256), (3, 16, 4096, 256),
    (4, 8, 4096, 256),
    (5, 8, 4096, 256), (6, 8, 4096, 256), (7, 8, 4096, 256), (8, 8, 4096, 256),
    (9, 8, 4096, 256),
    (10, 1, 4096, 256), (10, 2, 4096, 256), (10, 4, 4096, 256), (10, 8, 4096, 256),
    (10, 2, 512, 256), (10, 4, 512, 256), (10, 4, 256, 256), (10, 8, 256, 256),
    (11, 8, 4096, 256),
    (12, 2, 4096, 256), (12, 4, 4096, 256), (12, 8, 4096, 256), (12, 4, 1024, 256),
    (13, 1, 4096, 256), (13, 2, 4096, 256), (13, 4, 4096, 256), (13, 8, 4096, 256),
    (14, 16, 4096, 256), (15, 16, 4096, 256), (16, 16, 4096, 256), (17, 16, 4096, 256),
    (18, 16, 4096, 256), (19, 16, 4096, 256), (20, 16, 4096, 256),
]


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = [nbuild.hipcc(), *nbuild.HIPCC_FLAGS, "-shared", SRC, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


def run(reps: int = 5, clock_ghz: float = 2.4, target: float = 3e10):
    import torch

    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built; run build() first")
    lib = ctypes.CDLL(LIB)
    lib.mb_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.mb_run.restype = ctypes.c_int
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    most = max(b * t for _, _, b, t in CASES)
    out = torch.empty(most, dtype=torch.float32, device="cuda:0")
    rows = []
    for op, ilp, blocks, threads in CASES:
        name, per = OPS[op]
        iters = max(1, int(target / (blocks * threads * ilp * per)))
        ms = ctypes.c_double()
        st = lib.mb_run(op, ilp, ctypes.c_void_p(out.data_ptr()), blocks, threads, iters, reps,
                        ctypes.byref(ms))
        if st != 0:
            raise RuntimeError(f"mb_run({name}, ilp={ilp}) failed with {st}")
        lane_instr = float(blocks) * threads * iters * ilp * per
        rate = lane_instr / (ms.value * 1e-3)
        waves_per_simd = blocks * threads / 64 / (cus * 4)
        row = {"op": name, "ilp": ilp, "blocks": blocks, "threads": threads,
               "waves_per_simd": round(waves_per_simd, 2), "ms": round(ms.value, 4),
               "lane_instr_per_cu_clk": round(rate / (cus * clock_ghz * 1e9), 2)}
        if op in (10, 12, 13, 20):
            # each symmetric evaluation serves two interactions
            per_eval = 2 if op == 12 else 1
            evals = 16 if op == 12 else 1
            inter = float(blocks) * threads * iters * ilp * evals * per_eval / (ms.value * 1e-3)
            if op == 20:   # four pairs per iteration (ilp counts its 16 instruction slots)
                inter = float(blocks) * threads * iters * 4 / (ms.value * 1e-3)
            row["G_interactions_per_s"] = round(inter / 1e9, 1)
            row["pct_fp32_peak_at_20_flops"] = round(100 * 20 * inter / 157.3e12, 1)
        rows.append(row)
    return {"device": props.name, "cus": cus, "clock_ghz": clock_ghz, "cases": rows}


if __name__ == "__main__":
    import sys

    if "--no-build" not in sys.argv[1:]:   # the library built in-tree beforehand
        build()
    print(json.dumps(run()))
