"""Build libedpc.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2507_18969_amd.build [--jobs N]
Every translation unit under csrc/ is compiled to an object in _build/ and
linked into paper_2507_18969_amd/libedpc.so.

With --sanitize the host code (not the device code) is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer into _build/sanitize/libedpc.so,
for host-only tests run with the ASan runtime preloaded (EDPC_LIB names it).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libedpc.so")
SOURCES = ["gemm.hip", "gemm_wide.hip", "kernels.hip", "fused.hip", "model.hip", "codec.hip", "stream.hip", "ksg.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# roctx, for the named host-side ranges (csrc/trace.h) that profilers record
ROCTX_LINK = ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
              "-Wl,-rpath," + os.path.join(ROCM, "lib")]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions disabled for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


# host-side sanitizers only: every -fsanitize sits behind -Xarch_host, so the
# gfx950 code object is built exactly as in the product library
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_BUILD, "libedpc.so")


def asan_runtime() -> str:
    """Path of the compiler's ASan runtime (to preload into a host process)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    return r.stdout.strip()


# per-kernel register, scratch and LDS use of the product build, from the
# compiler's resource-usage remarks (one row per kernel)
RESOURCES = os.path.join(BUILD, "kernel_resources.tsv")
RESOURCE_FIELDS = [("VGPRs", "vgprs"), ("AGPRs", "agprs"), ("ScratchSize [bytes/lane]", "scratch"),
                   ("VGPRs Spill", "vgpr_spill"), ("SGPRs Spill", "sgpr_spill"),
                   ("LDS Size [bytes/block]", "lds"), ("Occupancy [waves/SIMD]", "occupancy")]
_REMARK = re.compile(r"remark:\s+(.+?): (.+?) \[-Rpass-analysis=kernel-resource-usage\]")


def _resources(src: str, stderr: str) -> list:
    rows, cur = [], None
    keys = dict(RESOURCE_FIELDS)
    for m in _REMARK.finditer(stderr):
        k, v = m.group(1).strip(), m.group(2).strip()
        if k == "Function Name":
            cur = {"source": src, "kernel": v}
            rows.append(cur)
        elif cur is not None and k in keys:
            cur[keys[k]] = v
    return rows


def _compile(src: str, sanitize: bool = False):
    out = SAN_BUILD if sanitize else BUILD
    obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
    remarks = [] if sanitize else ["-Rpass-analysis=kernel-resource-usage"]
    cmd = [HIPCC, *FLAGS, *(SANITIZE if sanitize else []), *remarks, "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj, _resources(src, r.stderr)


def _write_resources(rows: list) -> None:
    cols = ["source", "kernel"] + [c for _, c in RESOURCE_FIELDS]
    with open(RESOURCES + ".tmp", "w") as f:
        f.write("\t".join(cols) + "\n")
        for row in sorted(rows, key=lambda r: (r["source"], r["kernel"])):
            f.write("\t".join(str(row.get(c, "")) for c in cols) + "\n")
    os.replace(RESOURCES + ".tmp", RESOURCES)


def build(jobs: int = 5, verbose: bool = True, sanitize: bool = False) -> str:
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        done = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    objs = [o for o, _ in done]
    if not sanitize:
        _write_resources([row for _, rows in done for row in rows])
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *(SANITIZE if sanitize else []),
           *objs, *ROCTX_LINK, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=5)
    ap.add_argument("--sanitize", action="store_true",
                    help="host ASan + UBSan build into _build/sanitize/libedpc.so")
    a = ap.parse_args()
    try:
        build(a.jobs, sanitize=a.sanitize)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
