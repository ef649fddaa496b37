"""Compile libpdmi.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdmi.so")

SOURCES = ["geometry.cpp", "kl.cpp", "solver.hip", "static_batch.hip", "fields.hip", "adjoint.hip", "material.hip",
           "launch_f32_kahan.hip", "launch_f32_kahan_c.hip", "launch_f32_plain.hip", "launch_f64.hip"]

# the dense eigensolver of the exponential-covariance KL basis
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no implicit FMA contraction: fused operations are written out
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-fvisibility=hidden",
    "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def kernel_resources(remarks: str):
    """Per-kernel (VGPRs, spilled VGPRs, scratch bytes per lane, occupancy)
    from the compiler's kernel-resource-usage remarks."""
    import re
    out, name = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|VGPRs Spill|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)",
                      line)
        if m and name:
            key = {"VGPRs": "VGPRs", "VGPRs Spill": "VGPRSpill"}.get(m.group(1), m.group(1).split()[0])
            out[name][key] = int(m.group(2))
    return out


def resource_problems(res):
    """Step-kernel resource use that fails the build, from kernel_resources()
    output: FP32 step kernels that use scratch memory (spilled registers, or
    a private array not kept in registers; a scratch access in the exception
    pass's round loops costs a sixth of the cracking-load throughput), and
    FP32 kernels of the default 16x4x4 brick without a micromodulus tile that
    need more than 128 VGPRs (they hold 4 waves per SIMD only up to 128, the
    38.4 KB tile allowing no more; with the c tile, LDS caps them at 3
    anyway)."""
    import re
    out = []
    scratch = [k for k, v in res.items() if "step_kernelIf" in k and
               (v.get("VGPRSpill", 0) > 0 or v.get("ScratchSize", 0) > 0)]
    if scratch:
        out.append("FP32 step kernels use scratch memory: " + ", ".join(scratch))
    wide = [f"{k} ({v.get('VGPRs')} VGPRs)" for k, v in res.items()
            if re.search(r"step_kernelIfLb[01]ELb0ELb1ENS_5BrickILi16ELi4ELi4ELi2E", k) and v.get("VGPRs", 0) > 128]
    if wide:
        out.append("FP32 16x4x4 step kernels need more than 128 VGPRs: " + ", ".join(wide))
    return out


def _compile(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return r.stderr


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links.  The step
    kernels' resource use is read from the compiler's remarks, and what
    resource_problems() names fails the build."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="pdmi_build_") as tmpdir:
        objs, cmds = [], []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            extra = ["-Rpass-analysis=kernel-resource-usage"] if os.path.basename(src).startswith("launch_") else []
            cmds.append([HIPCC, *compile_flags, *extra, *inc, "-c", "-o", obj, src])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        # one hipcc per source, at most 16 at once (a shared host's CPU share)
        with ThreadPoolExecutor(max_workers=min(len(cmds), 16, max(1, os.cpu_count() or 1))) as ex:
            remarks = "".join(f.result() for f in [ex.submit(_compile, c) for c in cmds])
        res = {k: v for k, v in kernel_resources(remarks).items() if "step_kernel" in k}
        if verbose:
            for k, v in sorted(res.items()):
                print(f"{k}: {v}", flush=True)
        problems = resource_problems(res)
        if problems:
            raise RuntimeError("; ".join(problems))
        tmp = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(out: str) -> str:
    """The library with AddressSanitizer on its host code (-O1 -g) into
    `out`, for host checks of the entry points that run without a GPU (mesh
    and bond construction, argument checks, the MLMC allocation, bias and
    rate fit).  The device code is compiled as usual but never run from
    this build.  Load it with PDMI_LIB=<out> in a process that preloads
    sanitizer_runtime()."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
             "-fvisibility=hidden", "-Wno-unused-result",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with tempfile.TemporaryDirectory(prefix="pdmi_asan_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[HIPCC, *flags, *inc, "-c", "-o", o, src] for o, src in zip(objs, sources())]
        with ThreadPoolExecutor(max_workers=min(len(cmds), 16, max(1, os.cpu_count() or 1))) as ex:
            for f in [ex.submit(_compile, c) for c in cmds]:
                f.result()
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs, *LIBS])
    return out


def sanitizer_runtime() -> str:
    """The AddressSanitizer runtime of the compiler that built the library
    (to preload ahead of Python)."""
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    return found[-1]


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
