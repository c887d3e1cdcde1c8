"""Builds ``libnze.so`` (HIP for gfx950 + host C++) in the package folder."""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnze.so")

SOURCES = ["nze_mpo.hip", "nze_host.cpp", "nze_serve.cpp"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # no packed fp32 instructions on this target
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # per-kernel register, scratch and LDS figures on stderr
         "-Rpass-analysis=kernel-resource-usage"]

# Layer kernels that must run without a stack: every helper is inlined and
# nothing spills, so a launch touches no scratch memory.  (The kernel built
# for two workgroups per CU is capped at 256 registers and may spill.)
NO_SCRATCH = ("k_layer_f32E", "k_layer_f64E")


def resource_usage(stderr):
    """{mangled kernel name: {field: value}} from the compiler's
    kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return out


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    usage = resource_usage(res.stderr)
    for key in NO_SCRATCH:
        names = [n for n in usage if key in n]
        if not names:
            raise RuntimeError(f"no resource usage reported for {key}")
        for n in names:
            scratch = int(usage[n].get("ScratchSize [bytes/lane]", "-1"))
            if scratch != 0:
                os.remove(tmp)
                raise RuntimeError(f"{n} needs {scratch} bytes of scratch per lane "
                                   f"(a helper was not inlined or registers spilled)")
    if verbose:
        print(" ".join(cmd))
        for n, u in usage.items():
            if "k_layer" in n:
                print(n, {k: u.get(k) for k in ("VGPRs", "AGPRs", "ScratchSize [bytes/lane]",
                                                 "VGPRs Spill", "Occupancy [waves/SIMD]")})
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
