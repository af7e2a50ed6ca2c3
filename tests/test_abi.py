"""The C-ABI library loads and exports every function include/caf_gpu.h
declares; argument checks that happen before any device call."""
import ctypes as C
import os
import re

import pytest

from paper_1505_07368_amd import binding as cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "caf_gpu.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(caf_\w+)\s*\(", text, re.M)))


def test_header_declares_the_actor_calls():
    names = declared_functions()
    for required in ("caf_gpu_spawn", "caf_gpu_send", "caf_gpu_request", "caf_gpu_quit",
                     "caf_future_wait", "caf_gpu_init", "caf_gpu_shutdown"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = cg.load()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(cg.EXPORTED) == sorted(declared_functions())


def test_strerror_and_init_argument_checks():
    L = cg.load()
    assert L.caf_gpu_strerror(0) == b"ok"
    assert b"quit" in L.caf_gpu_strerror(cg.E_QUIT)
    h = C.c_void_p()
    cfg = cg.caf_gpu_config()  # NULL arena: rejected before touching a device
    assert L.caf_gpu_init(C.byref(cfg), C.byref(h)) == cg.E_INVALID
    assert L.caf_gpu_init(None, C.byref(h)) == cg.E_INVALID
    bogus = cg.caf_gpu_config()  # unknown mode: rejected before any device call
    bogus.arena = 1 << 40
    bogus.arena_bytes = 1 << 20
    bogus.mode = 4
    assert L.caf_gpu_init(C.byref(bogus), C.byref(h)) == cg.E_INVALID
    assert L.caf_gpu_spawn(None, 0, None, None) == cg.E_INVALID
    assert L.caf_gpu_quit(None, 1, 0) == cg.E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the header's structs have the C layout (sizes and
    field offsets from the header compiled by gcc)."""
    import subprocess
    structs = {"caf_buf": cg.caf_buf, "caf_gpu_config": cg.caf_gpu_config,
               "caf_mandel_args": cg.caf_mandel_args, "caf_gemm_args": cg.caf_gemm_args,
               "caf_shape_args": cg.caf_shape_args, "caf_hash_args": cg.caf_hash_args,
               "caf_spawn_args": cg.caf_spawn_args, "caf_gpu_stats": cg.caf_gpu_stats,
               "caf_msg": cg.caf_msg}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(){']
    for name, ct in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in ct._fields_:
            cf = "in" if f == "in_" else f
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.splitlines():
        name, field, val = line.split()
        ct = structs[name]
        got = C.sizeof(ct) if field == "size" else getattr(ct, field).offset
        assert got == int(val), (name, field, got, val)


def test_enum_values_match_header(tmp_path):
    """The binding's behaviour, mode and grouping constants equal the header's
    enumerators (compiled by gcc)."""
    import subprocess
    pairs = {"CAF_BHV_NOOP": cg.BHV_NOOP, "CAF_BHV_MANDELBROT": cg.BHV_MANDELBROT,
             "CAF_BHV_GEMM": cg.BHV_GEMM, "CAF_BHV_TANH": cg.BHV_TANH,
             "CAF_BHV_ROWSUM": cg.BHV_ROWSUM, "CAF_BHV_HASHCHAIN": cg.BHV_HASHCHAIN,
             "CAF_BHV_FAULT": cg.BHV_FAULT, "CAF_MODE_PLAIN": cg.MODE_PLAIN,
             "CAF_MODE_BATCHED": cg.MODE_BATCHED, "CAF_MODE_PERSISTENT": cg.MODE_PERSISTENT,
             "CAF_MODE_PLAIN_GRAPH": cg.MODE_PLAIN_GRAPH, "CAF_GROUP_FIFO": cg.GROUP_FIFO,
             "CAF_GROUP_LPT": cg.GROUP_LPT, "CAF_GROUP_KIND": cg.GROUP_KIND}
    lines = ['#include <stdio.h>', f'#include "{HEADER}"', 'int main(){']
    lines += [f'printf("{k} %d\\n", (int){k});' for k in pairs]
    lines.append("return 0;}")
    src = tmp_path / "enums.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "enums"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict((k, int(v)) for k, v in (l.split() for l in out.splitlines()))
    assert got == pairs
    assert set(cg.GROUPINGS.values()) == {cg.GROUP_FIFO, cg.GROUP_LPT, cg.GROUP_KIND}
