"""Build step: regenerate the per-process HIP code and compile libnlome.so
for gfx950 in-tree (one object per process and kernel variant, compiled in
parallel, then linked)."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnlome.so")
PROBE_LIB = os.path.join(HERE, "libnlome_probe.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are disabled on purpose (plain FP32 FMAs only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
]


# Per-unit overrides.  The BF16 variant of g g -> t tbar g g (an accuracy study:
# gfx950 has no BF16 arithmetic, so every operation is widened to FP32 and
# rounded back) takes 7.5 minutes to optimise at -O3, far longer than every
# other unit together, almost all of it in unrolling the short inner loops.
# Without loop unrolling it takes 2 minutes and runs 104 ms per 2^20 events
# (at -O1: 122 ms; fully unrolled at -O3: 62.5 ms).
UNIT_FLAGS = {"tu_gg_ttgg_4.hip": ("-fno-unroll-loops",)}

# |M|^2 units in FP64, FP32 and with MFMA colour (tu_<process>_<0|1|2>.hip,
# and 5, 6 for the alternative helicity schedule in FP64 and FP32):
# external polarisation vectors have a zero time component and a real z
# component, and massless spinors have a zero chiral half.  Under strict IEEE
# rules the compiler must keep every product with those zeros (x * 0 is NaN
# for infinite x and -0 for negative x); these kernels test no value for NaN
# or infinity and never produce one from finite momenta, so they drop those
# rules and the products fold away (about 11 % fewer instructions for
# g g -> t tbar g).  The FP16/BF16 units (3, 4) keep infinities: they route an
# event with an infinite propagator factor to the FP32 pass.  The FKS units
# keep full IEEE semantics: they test the subtracted weight for finiteness.
ME2_FAST_FLAGS = {"0": ("-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros"),
                  "1": ("-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros"),
                  "2": ("-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros"),
                  "3": ("-fno-honor-nans", "-fno-signed-zeros"),
                  "4": ("-fno-honor-nans", "-fno-signed-zeros"),
                  "5": ("-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros"),
                  "6": ("-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros")}


def unit_flags(base):
    flags = list(UNIT_FLAGS.get(base, ()))
    if base.startswith("tu_") and not base.startswith("tu_fks_"):
        flags += ME2_FAST_FLAGS.get(os.path.splitext(base)[0].rsplit("_", 1)[1], ())
    return flags


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def generate():
    sys.path.insert(0, ROOT)
    from paper_2503_07439_amd import codegen
    return codegen.generate(os.path.join(CSRC, "generated"))


def _deps(src):
    """Sources an object depends on: the unit, the shared headers and, for a
    process unit, its generated header."""
    deps = [src] + [os.path.join(CSRC, h) for h in ("helas.hpp", "opaque.hpp", "kernels.hpp", "launch.hpp", "fks.hpp",
                                                     "phase_space.hpp", "checks.hpp")]
    deps.append(os.path.join(ROOT, "include", "nlome.h"))
    base = os.path.basename(src)
    if base.startswith("tu_fks_"):
        stem = base[3:].rsplit("_", 1)[0]
        deps.append(os.path.join(os.path.dirname(src), stem + ".hpp"))
        real = stem[4:].rsplit("_", 2)[0]
        deps.append(os.path.join(os.path.dirname(src), real + ".hpp"))
    elif base.startswith("tu_"):
        deps.append(os.path.join(os.path.dirname(src), base[3:].rsplit("_", 1)[0] + ".hpp"))
    else:
        deps.append(os.path.join(CSRC, "generated", "index.hpp"))
    return deps


def build_id():
    """A hash of every source the library is built from (the key that ties a
    tuning-cache entry to this build)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp")) +
                   glob.glob(os.path.join(CSRC, "generated", "*.hpp")))
    files += [os.path.join(ROOT, "include", "nlome.h"), os.path.join(HERE, "build.py"), os.path.join(HERE, "codegen.py")]
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src, extra, verbose, force, bid=None):
    obj = os.path.join(OBJ, os.path.splitext(os.path.basename(src))[0] + ".o")
    extra = list(extra)
    if bid is not None and os.path.basename(src) == "capi.hip":
        extra.append('-DNLO_BUILD_ID="%s"' % bid)
        stamp = os.path.join(OBJ, "capi.build_id")
        if not os.path.exists(stamp) or open(stamp).read() != bid:
            force = True
            with open(stamp, "w") as f:
                f.write(bid)
    if not force and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(os.path.getmtime(d) <= t for d in _deps(src) if os.path.exists(d)):
            return obj
    cmd = [_hipcc()] + HIPCC_FLAGS + extra + unit_flags(os.path.basename(src)) + ["-c", "-o", obj, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    if verbose:
        print("  built", os.path.basename(obj), flush=True)
    return obj


def build(verbose=True, extra_flags=(), jobs=None, force=True):
    """Compile every unit (force=True) or only those older than their sources."""
    tus = generate()
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, "capi.hip"), os.path.join(CSRC, "phase_space.hip"), os.path.join(CSRC, "checks.hip")] + list(tus)
    # the largest process first so the long poles start early
    srcs.sort(key=lambda p: 0 if p.endswith(("tu_gg_ttgg_4.hip", "tu_gg_ttgg_5.hip", "tu_gg_ttgg_6.hip")) else
              (1 if ("gg_ttgg" in p and "fks" not in p) else (2 if "gg_ttg" in p else 3)))
    jobs = jobs or min(16, os.cpu_count() or 8)
    bid = build_id()
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra_flags, verbose, force, bid), srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("linked", LIB, flush=True)
    build_probe()
    count_flops(verbose)
    return LIB


def build_probe():
    """The FMA-throughput probe the benchmark uses to quote the attainable
    vector-ALU peak (a library of its own: no part of the C ABI)."""
    src = os.path.join(CSRC, "probe.hip")
    tmp = PROBE_LIB + ".tmp"
    cmd = [_hipcc()] + HIPCC_FLAGS + ["-shared", "-o", tmp, src]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def count_flops(verbose=True):
    """Compile and run the host operation counter; writes flops.json (the
    algorithmic flop count per event used for the roofline)."""
    exe = os.path.join(OBJ, "opcount")
    src = os.path.join(CSRC, "opcount.hip")
    cmd = [_hipcc(), "-O0", "-std=c++17", "--offload-arch=gfx950", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           "-o", exe, src]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    import json
    data = json.loads(out)
    with open(os.path.join(HERE, "flops.json"), "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    if verbose:
        print("flop counts written", flush=True)
    return data


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv)
