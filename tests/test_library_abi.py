"""CPU checks of the C ABI: the library loads, exports every function that
include/pdhcg.h declares, and returns the documented defaults (no GPU work)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="pdhcg.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhcg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ["pdhcg_create", "pdhcg_solve", "pdhcg_solve_batch", "pdhcg_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_16160_amd import pdhcg
    L = pdhcg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(pdhcg.EXPORTS)


def test_library_exports_the_network_abi():
    from paper_2405_16160_amd import mlp, pdhcg
    L = pdhcg.lib()
    names = declared_functions("pdhcg_mlp.h")
    assert set(names) == set(mlp.MLP_EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def test_default_settings_match_the_paper_constants():
    from paper_2405_16160_amd import pdhcg
    s = pdhcg.default_settings()
    assert s.cg_eps_factor == 0.05
    assert (s.beta_sufficient, s.beta_necessary, s.beta_artificial) == (0.2, 0.8, 0.2)
    assert s.primal_weight_theta == 0.2
    assert s.step_eta_factor == 0.5
    assert s == pdhcg.Settings()


def test_error_strings():
    from paper_2405_16160_amd import pdhcg
    L = pdhcg.lib()
    assert L.pdhcg_error_string(-1) == b"invalid argument"
    assert L.pdhcg_error_string(-3) == b"HIP error"


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every field of the ctypes mirrors sits at the offset the C compiler gives
    it in include/pdhcg.h, and each struct has the header's size (a C program
    built with gcc prints sizeof and offsetof)."""
    import ctypes as C
    import subprocess
    from paper_2405_16160_amd import pdhcg
    structs = [pdhcg.pdhcg_csr, pdhcg.pdhcg_settings, pdhcg.pdhcg_lowrank, pdhcg.pdhcg_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdhcg.h"', "int main(void) {"]
    for st in structs:
        t = st.__name__
        lines.append(f'  printf("{t} sizeof %zu\\n", sizeof({t}));')
        for name, _ in st._fields_:
            lines.append(f'  printf("{t} {name} %zu\\n", offsetof({t}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        t, name, v = line.split()
        got[(t, name)] = int(v)
    for st in structs:
        t = st.__name__
        assert got[(t, "sizeof")] == C.sizeof(st), t
        for name, _ in st._fields_:
            assert got[(t, name)] == getattr(st, name).offset, (t, name)
