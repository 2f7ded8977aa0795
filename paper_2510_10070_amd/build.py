"""Build the HIP library libsbp.so in-tree for gfx950 (hipcc, no JIT).

Variants (python -m paper_2510_10070_amd.build [--variant V]):
  default  libsbp.so, the product;
  poison   libsbp_poison.so: every kernel fills its shared arrays with NaN before first use
           (SBP_POISON_LDS), so that a read of LDS no thread wrote shows up in the parity tests;
  asan     libsbp_asan.so: the host-side translation units (plan, validation, tables, tuner,
           launchers) built with AddressSanitizer for the host only, linked with the default
           build's kernel objects; load it with the sanitizer runtime preloaded.
The binding loads a variant when SBP_LIBRARY_VARIANT names it (default: the product).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["sbp_plan.hip", "tune.hip", "dispatch.hip", "plain.hip", "pass_y_f32.hip", "pass_y_f64.hip",
           "pass_x_f32.hip", "pass_x_f64.hip", "pass_z_f32.hip", "pass_z_f64.hip",
           "fused_f32.hip", "fused_f64.hip", "gravity.hip"]
# fused passes A and C, split by Ny so that they compile in parallel
SOURCES += [f"fused_{p}_{y}.hip" for p in ("f32", "f64") for y in ("y16_64", "y96_128", "y256", "y512")]
SOURCES += ["fused_f32_multi.hip", "fused_f32_multi_b.hip", "fused_f32_wide_ac.hip", "fused_f32_wide_b.hip"]
# translation units whose host code the sanitizer build instruments
HOST_SOURCES = ["sbp_plan.hip", "tune.hip", "dispatch.hip", "plain.hip", "gravity.hip"]

VARIANTS = {
    "default": dict(lib="libsbp.so", build="_build", flags=[]),
    "poison": dict(lib="libsbp_poison.so", build="_build_poison", flags=["-DSBP_POISON_LDS"]),
    "asan": dict(lib="libsbp_asan.so", build="_build_asan",
                 flags=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]),
}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "--offload-arch=gfx950",
    # never emit packed FP32 arithmetic: the compiler forms it from scalar/float2 code otherwise
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(src: str, build_dir: str, extra) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, variant: str = "default") -> str:
    v = VARIANTS[variant]
    build_dir = os.path.join(HERE, v["build"])
    lib = os.path.join(HERE, v["lib"])
    os.makedirs(build_dir, exist_ok=True)
    if variant == "asan":
        # instrumented host translation units, everything else from the default build
        base = os.path.join(HERE, VARIANTS["default"]["build"])
        missing = [s for s in SOURCES if s not in HOST_SOURCES
                   and not os.path.exists(os.path.join(base, s.replace(".hip", ".o")))]
        if missing:
            raise RuntimeError(f"the sanitizer build links the default build's objects; build that first ({missing[0]})")
        srcs = HOST_SOURCES
    else:
        srcs = SOURCES
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, v["flags"]), srcs))
    if variant == "asan":
        objs += [os.path.join(base, s.replace(".hip", ".o")) for s in SOURCES if s not in HOST_SOURCES]
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address"] if variant == "asan" else []
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *link_extra, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--variant", choices=sorted(VARIANTS), default="default")
    build(verbose=True, variant=ap.parse_args().variant)
    sys.exit(0)
