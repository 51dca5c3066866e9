"""Build libapax.so (HIP for gfx950) in-tree with hipcc."""
import concurrent.futures as cf
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libapax.so")
SOURCES = ["capi.hip", "encode.hip", "decode.hip", "profile.hip", "batch_enc.hip", "batch_dec.hip",
           "s2r.hip", "spectra.hip", "monitor.hip", "wide.hip", "adapt.hip", "profile_wide.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-I", INC, "-I", CSRC, "-Wall", "-Wno-unused-function"]
LLVM = "/opt/rocm/llvm/bin"
# A DPP lane move folded into a subtraction (v_sub*_dpp / v_subrev*_dpp) gave
# negated results on gfx950, so the sources only ever add a shifted operand
# (a shifted difference is sent negated); every object is checked for it.
BAD_DPP = re.compile(r"\bv_sub(?:rev)?[a-z0-9_]*_dpp\b")


def _check_dpp(obj):
    """Disassemble the gfx950 code object of `obj` and refuse subtract-DPP forms."""
    with tempfile.TemporaryDirectory() as td:
        fat, co = os.path.join(td, "fat"), os.path.join(td, "co")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f".hip_fatbin={fat}", obj],
                       check=True, capture_output=True)
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                        f"--input={fat}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                       check=True, capture_output=True)
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", co], check=True,
                             capture_output=True, text=True).stdout
    bad = sorted(set(BAD_DPP.findall(dis)))
    if bad:
        raise RuntimeError(f"{os.path.basename(obj)}: subtract-DPP instructions {bad}; "
                           "write the shifted operand as an added negation")
    # A DPP lane move reads zero from lanes that are switched off, so none
    # may run while a divergent branch has narrowed the execution mask: scan
    # each function in order, tracking whether the last write of exec narrowed
    # it (saveexec / and / andn2 / xor) or restored it (or / mov); code after
    # an unconditional branch starts a block reached by jumps only, whose mask
    # this scan does not follow.
    narrowed, where = False, []
    for line in dis.splitlines():
        t = line.split("//")[0].strip()
        if t.endswith(">:"):
            narrowed = False
            continue
        ops = t.split()
        op = next((o for o in ops if o.startswith(("s_", "v_"))), None)
        if op is None:
            continue
        if op in ("s_branch", "s_endpgm", "s_setpc_b64"):
            narrowed = False
        elif op.startswith(("s_and_saveexec", "s_andn2_saveexec", "s_xor_saveexec")) or \
                (op.startswith(("s_and_b64", "s_andn2_b64", "s_xor_b64")) and "exec," in t.split(op, 1)[1][:8]):
            narrowed = True
        elif op.startswith(("s_or_b64", "s_or_saveexec", "s_mov_b64")) and "exec" in t.split(op, 1)[1][:8]:
            narrowed = False
        elif "_dpp" in op and narrowed:
            where.append(t)
    if where:
        raise RuntimeError(f"{os.path.basename(obj)}: DPP under a narrowed exec mask: {where[:4]}")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    _check_dpp(obj)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
