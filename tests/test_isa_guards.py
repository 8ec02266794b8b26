"""Guards on the machine code of the built library (gfx950 code objects of
libsncc.so, disassembled with the ROCm LLVM tools; no GPU needed).

On gfx950 the folded form v_subrev_u32_dpp d, a, b (which the compiler emits
for b - shr(a)) computes shr(b) - a: the shift lands on the other operand (a
one-wave probe with distinct registers showed it).  No kernel may contain an
operand-reversed VOP2 op with a DPP source, and the slow pass and the refine
kernel, whose slot loops take no value from another lane (summation by
parts over the segments' corners), may contain no subtraction with a
row-shifted DPP source.  A compiler change that folds such an operation fails here, on the
CPU, before any GPU run.
"""

import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2502_01286_amd", "libsncc.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def _disassembly():
    objcopy, bundler, objdump = (_tool("llvm-objcopy"), _tool("clang-offload-bundler"),
                                 _tool("llvm-objdump"))
    if not (objcopy and bundler and objdump and os.path.exists(LIB)):
        pytest.skip("ROCm LLVM tools or the built library not available")
    out = []
    with tempfile.TemporaryDirectory() as d:
        fb = os.path.join(d, "fatbin")
        subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fb}", LIB], check=True)
        data = open(fb, "rb").read()
        starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)] + [len(data)]
        for i, (a, b) in enumerate(zip(starts, starts[1:])):
            part = os.path.join(d, f"b{i}")
            with open(part, "wb") as fh:
                fh.write(data[a:b])
            co = os.path.join(d, f"b{i}.co")
            r = subprocess.run([bundler, "--unbundle", "--type=o", f"--input={part}",
                                "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                               capture_output=True)
            if r.returncode != 0 or not os.path.getsize(co):
                continue
            r = subprocess.run([objdump, "-d", "--mcpu=gfx950", co], capture_output=True,
                               text=True, check=True)
            out.append(r.stdout)
    return "\n".join(out)


def _functions(text):
    """Disassembly split by function symbol: {mangled name: body}."""
    funcs, name, body = {}, None, []
    for line in text.splitlines():
        m = re.match(r"^[0-9a-f]+ <(.+)>:$", line)
        if m:
            if name:
                funcs[name] = "\n".join(body)
            name, body = m.group(1), []
        elif name:
            body.append(line)
    if name:
        funcs[name] = "\n".join(body)
    return funcs


def test_no_row_shifted_subtractions_in_the_fp64_slot_loops():
    funcs = _functions(_disassembly())
    kernels = {n: b for n, b in funcs.items()
               if "slow_kernel" in n or "refine_kernel" in n}
    assert kernels, "slow_kernel / refine_kernel not found in the code objects"
    for name, body in kernels.items():
        folded = [ln for ln in body.splitlines()
                  if re.search(r"v_sub(rev)?_u32_dpp", ln) and "row_shr" in ln]
        assert not folded, (name, folded[:3])


def test_no_operand_reversed_dpp_ops_anywhere():
    funcs = _functions(_disassembly())
    assert funcs
    bad = [(n, ln.strip()) for n, b in funcs.items() for ln in b.splitlines()
           if re.search(r"\bv_\w*rev\w*_dpp\b", ln)]
    assert not bad, bad[:3]
