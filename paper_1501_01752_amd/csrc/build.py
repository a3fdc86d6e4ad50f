#!/usr/bin/env python3
"""Build libgsm.so for gfx950 in-tree: generate the FFT codelets, compile each
translation unit with hipcc in parallel and link the shared library next to
the Python package.  Usage: python build.py [--jobs N] [--out PATH] [-D NAME=VALUE ...]
(--out and -D build a variant library elsewhere, e.g. for comparing kernel
settings; the package loads it when GSM_LIBRARY names it)."""
import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
BUILD = os.path.join(PKG, "_build")
UNITS = ["tu_passes_f32.hip", "tu_passes_f64.hip", "tu_krylov.hip", "tu_plan.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         # packed FP32 instructions stay out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise SystemExit(f"build failed: {cmd[-1]}")
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(PKG, "libgsm.so"))
    ap.add_argument("-D", dest="defines", action="append", default=[])
    args = ap.parse_args()
    build = BUILD if not args.defines else os.path.join(BUILD, "variant_" + "_".join(
        d.replace("=", "-") for d in args.defines))
    os.makedirs(build, exist_ok=True)
    flags = FLAGS + ["-D" + d for d in args.defines]
    if args.defines:
        # a variant gets codelets of its own (the generator reads its options
        # from the environment), so the default build's header stays as it is
        header = os.path.join(build, "fft_codelets.h")
        run([sys.executable, os.path.join(HERE, "gen_fft.py"), header])
        flags.append(f'-DGSM_CODELETS="{header}"')
    else:
        run([sys.executable, os.path.join(HERE, "gen_fft.py"), os.path.join(HERE, "fft_codelets.h")])

    def compile_unit(u):
        obj = os.path.join(build, u.replace(".hip", ".o"))
        run([HIPCC] + flags + ["-c", os.path.join(HERE, u), "-o", obj])
        return obj

    with ThreadPoolExecutor(args.jobs) as ex:
        objs = list(ex.map(compile_unit, UNITS))
    out = os.path.abspath(args.out)
    tmp = out + ".tmp"
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    print(out)


if __name__ == "__main__":
    main()
