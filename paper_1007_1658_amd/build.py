"""Build libmi355lsp.so (HIP for gfx950 + host C++) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 code generation
turned off (-packed-fp32-ops): the kernels are written in plain scalar FP32.
"""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmi355lsp.so")
SOURCES = ["pgram_kernels.hip", "pgram_mfma.hip", "batch_kernels.hip", "mlp_kernels.hip", "microbench.hip", "probe_kernels.hip", "fast_kernels.hip", "noalloc.hip", "fast_host.cpp", "lsp_host.cpp",
           "tuner.cpp", "surrogate.cpp"]
ARCH = os.environ.get("LSP_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]
DEVICE = [
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str, verbose: bool, defines=()) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    obj = os.path.join(OUT_DIR, src + (".poison" if defines else "") + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + list(defines)
    if src.endswith(".hip"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    return obj


POISON_SRC = "pgram_mfma.hip"   # the kernels whose waves share LDS operands across barriers
POISON_LIB = os.path.join(PKG, "debug", "libmi355lsp_poison.so")


def build(verbose: bool = False) -> str:
    jobs = [(s, ()) for s in SOURCES] + [(POISON_SRC, ("-DLSP_POISON_LDS",))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], verbose, j[1]), jobs))
    main_objs, poison_obj = objs[:len(SOURCES)], objs[len(SOURCES)]
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + main_objs + ["-lhipfft"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    # debug variant: shared LDS operands poisoned with NaN between blocks (race check)
    os.makedirs(os.path.dirname(POISON_LIB), exist_ok=True)
    pobjs = [poison_obj if s == POISON_SRC else o for s, o in zip(SOURCES, main_objs)]
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", POISON_LIB + ".tmp"] + pobjs + ["-lhipfft"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(POISON_LIB + ".tmp", POISON_LIB)
    build_cli(verbose)
    build_host_check(verbose)
    return LIB


HOST_SOURCES = ["lsp_host.cpp", "tuner.cpp", "surrogate.cpp", "fast_host.cpp"]
CHECK_DIR = os.path.join(OUT_DIR, "host_check")
CHECK = os.path.join(CHECK_DIR, "host_check")
# host C++ only, built with the plain clang++ of ROCm (no HIP mode, no device code)
SANITIZE = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def build_host_check(verbose: bool = False) -> str:
    """The host sources under AddressSanitizer/UBSan, linked with the device
    objects of the main build and tests/host_check.cpp (validation paths and
    file parsers, no GPU needed)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cxx = os.path.join(rocm, "llvm", "bin", "clang++")
    os.makedirs(CHECK_DIR, exist_ok=True)
    base = [cxx, "-x", "c++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-Wno-unused-value",
            "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + SANITIZE
    jobs = [(os.path.join(CSRC, f), os.path.join(CHECK_DIR, f + ".o")) for f in HOST_SOURCES]
    jobs.append((os.path.join(ROOT, "tests", "host_check.cpp"), os.path.join(CHECK_DIR, "host_check.o")))

    def one(job):
        cmd = base + ["-c", job[0], "-o", job[1]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return job[1]

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        objs = list(ex.map(one, jobs))
    dev = [os.path.join(OUT_DIR, f + ".o") for f in SOURCES if f.endswith(".hip")]
    cmd = [cxx] + SANITIZE + objs + dev + ["-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-lhipfft",
                                           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", CHECK + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CHECK + ".tmp", CHECK)
    return CHECK


CLI_SRC = os.path.join(PKG, "cli", "lsp_run.c")
CLI = os.path.join(PKG, "cli", "lsp_run")


def build_cli(verbose: bool = False) -> str:
    """lsp_run: a plain C program on the C ABI (include/lsp.h compiled as C11)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = [os.environ.get("CC", "gcc"), "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"), CLI_SRC,
           "-L" + PKG, "-lmi355lsp", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", CLI + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CLI + ".tmp", CLI)
    return CLI


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
