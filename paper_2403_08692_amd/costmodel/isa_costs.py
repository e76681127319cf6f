"""VALU issue-slot cost of each arithmetic building block, read from the
gfx950 assembly of isa_probe.hip (compiled here with the library's flags).

A VALU instruction of a wave64 occupies one SIMD for 4 cycles at full rate;
quarter-rate instructions (32-bit integer multiplies, 64-bit integer
multiply-adds, FP32/FP64 transcendental approximations and the FP64 trig
pre-op) occupy it four times as long.  The cost of a block is the weighted
VALU count of its probe kernel minus that of the probe's baseline (loads and
stores only).  Usage:  python -m paper_2403_08692_amd.costmodel.isa_costs
"""
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
QUARTER = re.compile(r"^v_(mul_lo_u32|mul_hi_u32|mul_hi_i32|mul_lo_i32|mad_u64_u32|mad_i64_i32|"
                     r"rcp_f64|rsq_f64|sqrt_f64|rcp_f32|rsq_f32|sqrt_f32|exp_f32|log_f32|sin_f32|"
                     r"cos_f32|trig_preop_f64|rcp_iflag_f32)\b")


def kernel_counts(asm: str):
    """Per probe kernel: [VALU instructions, issue slots, issue slots of the
    FP64 instructions (mnemonics with an _f64 operand type)]."""
    out = {}
    cur = None
    for line in asm.splitlines():
        m = re.match(r"^(probe_\w+):", line)
        if m:
            cur = m.group(1)
            out[cur] = [0, 0, 0]
            continue
        if cur is None:
            continue
        if line.strip().startswith("s_endpgm"):
            cur = None
            continue
        ins = line.strip().split(" ")[0]
        if ins.startswith("v_"):
            w = 4 if QUARTER.match(ins) else 1
            out[cur][0] += 1
            out[cur][1] += w
            if "_f64" in ins:
                out[cur][2] += w
    return out


def measure(fp64: bool = False):
    """Issue-slot cost per lane of each building block; with fp64, only its
    FP64 instructions (the FP64 roofline's count)."""
    sys.path.insert(0, os.path.dirname(HERE))
    from build import FLAGS, HIPCC  # noqa: E402

    flags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as d:
        s = os.path.join(d, "probe.s")
        subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", os.path.join(HERE, "isa_probe.hip"), "-o", s],
                       check=True, stderr=subprocess.DEVNULL)
        asm = open(s).read()
    c = kernel_counts(asm)
    col = 2 if fp64 else 1
    base = c["probe_base"][col]
    costs = {}
    for k, v in c.items():
        name = k[len("probe_"):]
        if name in ("base", "philox_base", "unit_base"):
            continue
        ref = base
        if name == "philox":
            ref = c["probe_philox_base"][col]
        if name == "unit":
            ref = c["probe_unit_base"][col]
        costs[name] = max(v[col] - ref, 0 if fp64 else 1)
    return costs


if __name__ == "__main__":
    print(json.dumps({"all": measure(), "fp64": measure(fp64=True)}, indent=1, sort_keys=True))
