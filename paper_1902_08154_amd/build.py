"""Build the gfx950 library libqp_pt2.so in-tree with hipcc.

Usage: python -m paper_1902_08154_amd.build   (or call build()).
Objects go to paper_1902_08154_amd/_build/; the shared library is written next
to this file, where the Python binding loads it.

Every kernel of the library must compile without scratch memory.  The kernels
have no private arrays that need it, so scratch use means register spills, and
the ROCm 7.2 compiler was seen to place a VGPR spill store at the start of a
join block before the EXEC mask was restored: the spill then covered only
some lanes and a value reloaded later was wrong for the others.  The build
reads the compiler's resource-usage remarks; when a dense-sweep instantiation
spills, its entry in csrc/qp_fast_caps.h (the occupancy its register
allocation aims for) is lowered and that source recompiled.  Any other kernel
that uses scratch fails the build.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqp_pt2.so")
SOURCES = ["qp_core.hip", "qp_sweep.hip", "qp_fast_fwd.hip", "qp_fast_bwd.hip"]
FAST_SOURCES = {"qp_fast_fwd.hip", "qp_fast_bwd.hip"}
CAPS = os.path.join(CSRC, "qp_fast_caps.h")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-munsafe-fp-atomics",
    # keep the compiler's own packed-FP32 selection off (see design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-Rpass-analysis=kernel-resource-usage",
]

_REMARK = re.compile(r"Function Name: (\S+)[\s\S]*?ScratchSize \[bytes/lane\]: (\d+)")
_FAST = re.compile(r"fast_kernelILi(\d)ELi(\d)ELb(\d)ELb(\d)E")


def _compile(src: str) -> tuple[str, dict[str, int]]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        err = "\n".join(l for l in res.stderr.splitlines() if "remark:" not in l)
        raise RuntimeError(f"hipcc failed for {src}:\n{err[-6000:]}")
    found = {m.group(1): int(m.group(2)) for m in _REMARK.finditer(res.stderr)}
    if not found:
        raise RuntimeError(f"hipcc printed no resource-usage remarks for {src}")
    return obj, found


def _read_caps() -> list:
    """caps[adjoint][fingerprint][n_int - 1][n_states - 1]"""
    txt = open(CAPS).read()
    body = txt[txt.index("= {") + 2: txt.rindex("};") + 1]
    nums = [int(x) for x in re.findall(r"\d+", body)]
    if len(nums) != 64:
        raise RuntimeError(f"{CAPS}: expected 64 entries, found {len(nums)}")
    return [[[nums[b * 32 + f * 16 + i * 4: b * 32 + f * 16 + i * 4 + 4] for i in range(4)] for f in range(2)]
            for b in range(2)]


def _write_caps(caps: list) -> None:
    txt = open(CAPS).read()
    head = txt[: txt.index("= {") + 3]

    def plane(b, f):
        return "{" + ", ".join("{" + ", ".join(str(v) for v in caps[b][f][i]) + "}" for i in range(4)) + "}"

    rows = [f"    {{{plane(b, 0)},\n     {plane(b, 1)}}}," for b in range(2)]
    open(CAPS, "w").write(head + "\n" + "\n".join(rows) + "\n};\n")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    todo = list(SOURCES)
    objs: dict[str, str] = {}
    for _ in range(8):
        with ThreadPoolExecutor(max_workers=len(todo)) as ex:
            results = dict(zip(todo, ex.map(_compile, todo)))
        caps = _read_caps()
        lowered = False
        bad = []
        spilling = {}
        for src, (obj, scratch) in results.items():
            objs[src] = obj
            for fn, size in scratch.items():
                if size == 0:
                    continue
                m = _FAST.search(fn)
                if m is None:
                    bad.append(f"{fn} ({size} bytes/lane)")
                    continue
                key = (int(m.group(3)), int(m.group(4)), int(m.group(1)), int(m.group(2)))
                spilling.setdefault(key, []).append((fn, size))
        for (bwd, fp, ni, ns), fns in spilling.items():
            if caps[bwd][fp][ni - 1][ns - 1] > 1:
                caps[bwd][fp][ni - 1][ns - 1] -= 1
                lowered = True
            else:
                bad += [f"{fn} ({size} bytes/lane at the lowest occupancy target)" for fn, size in fns]
        if bad:
            raise RuntimeError("kernels use scratch memory (register spills):\n  " + "\n  ".join(bad))
        if not lowered:
            break
        _write_caps(caps)
        if verbose:
            print("lowered occupancy targets in qp_fast_caps.h; recompiling the dense sweep", flush=True)
        todo = sorted(FAST_SOURCES)
    else:
        raise RuntimeError("occupancy targets did not settle")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[objs[s] for s in SOURCES], "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
