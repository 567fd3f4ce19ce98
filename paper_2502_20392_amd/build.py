"""Build libsigk.so (HIP, gfx950) in-tree.

Every (edge order P, channel bucket D) kernel variant listed in
csrc/sigk_internal.h is compiled from the same source in its own translation
unit (in parallel), then everything is linked into ``libsigk.so`` next to
this file.  ``build(force=False)`` reuses objects whose inputs are unchanged;
``build(force=True)`` recompiles everything.
"""
import concurrent.futures as cf
import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.environ.get("SIGK_OUT") or os.path.join(HERE, "libsigk.so")
BUILD = os.environ.get("SIGK_BUILD_DIR") or os.path.join(ROOT, "_build")

ARCH = os.environ.get("SIGK_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
EXTRA = os.environ.get("SIGK_EXTRA_FLAGS", "").split()
FLAGS = EXTRA + ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-I", INCLUDE]
HEADERS = ["sigk_internal.h", "sigk_device.h", "sigk_strip.h", "sigk_adjoint.h"]


def _variants(name):
    text = open(os.path.join(CSRC, "sigk_internal.h")).read()
    m = re.search(r"#define " + name + r"\(X\)((?:.*\\\n)*.*)", text)
    return [(int(p), int(d)) for p, d in re.findall(r"X\((\d+),\s*(\d+)\)", m.group(1))]


def _digest(paths, extra):
    h = hashlib.sha256()
    for p in paths:
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    h.update(repr(extra).encode())
    return h.hexdigest()[:16]


# Machine scheduler per translation unit.  Kernels that run one wave per SIMD
# (no other wave to hide a dependency's latency behind) gain from the
# iterative ILP scheduler: on the MMD^2 batch at order 10 the checkpointing
# sweep ran 6.6% and the adjoint 2.4% faster.  Where three waves share a SIMD
# (the forward at orders <= 6 with d <= 8) the default scheduler is faster
# (the order-5 long pair ran 2-4% slower with it), and the order-5 adjoint was
# unchanged.  The adjoint units keep the default from order 16 up, where this
# compiler's iterative scheduler fails on some of them.
ILP_SCHED = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]


def _unit_flags(src, defs):
    d = dict(defs)
    P, D = d.get("SIGK_P"), d.get("SIGK_D")
    if P is None:
        return []
    if src == "sigk_fwd.hip":
        return [] if (P <= 6 and D <= 8) else ILP_SCHED
    if src == "sigk_bwd.hip":
        return ILP_SCHED if 6 <= P <= 12 or (P <= 5 and D > 8) else []
    return []


def _compile(src, obj, defs, force):
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in HEADERS] + \
        [os.path.join(INCLUDE, "sigk.h")]
    flags = FLAGS + _unit_flags(src, defs)
    key = _digest(deps, (flags, defs, HIPCC))
    stamp = obj + ".key"
    if not force and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key:
        return obj
    cmd = [HIPCC, *flags, *[f"-D{k}={v}" for k, v in defs], "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {defs}:\n{r.stderr[-4000:]}")
    open(stamp, "w").write(key)
    return obj


def build(force: bool = False, jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [("sigk_api.hip", "api.o", []), ("sigk_static.hip", "static.o", []),
             ("sigk_estimate.hip", "estimate.o", []), ("sigk_delta.hip", "delta.o", [])]
    for p, d in _variants("SIGK_FWD_VARIANTS"):
        units.append(("sigk_fwd.hip", f"fwd_{p}_{d}.o", [("SIGK_P", p), ("SIGK_D", d)]))
    for p, d in _variants("SIGK_FWD_VARIANTS"):
        units.append(("sigk_fwd.hip", f"fwdt_{p}_{d}.o",
                      [("SIGK_P", p), ("SIGK_D", d), ("SIGK_ALT", 1)]))
    for p, d in _variants("SIGK_FWDG_VARIANTS"):
        units.append(("sigk_fwd.hip", f"fwd_{p}_{d}.o", [("SIGK_P", p), ("SIGK_D", d)]))
    for p, d in _variants("SIGK_FWDSQ_VARIANTS"):
        units.append(("sigk_fwd.hip", f"fwdsq_{p}_{d}.o",
                      [("SIGK_P", p), ("SIGK_D", d), ("SIGK_SQ", 1)]))
    for p, d in _variants("SIGK_BWD_VARIANTS"):
        units.append(("sigk_bwd.hip", f"bwd_{p}_{d}.o", [("SIGK_P", p), ("SIGK_D", d)]))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, src, os.path.join(BUILD, obj), defs, force)
                for src, obj, defs in units]
        objs = [f.result() for f in futs]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(objs)} objects")
    return OUT


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
