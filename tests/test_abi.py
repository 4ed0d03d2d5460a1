"""The C-ABI library loads on the CPU and exports every symbol that
include/ms2.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

from paper_1507_07548_amd import ms2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ms2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ms2_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["ms2_forces", "ms2_ewald_kspace", "ms2_step", "ms2_sample", "ms2_create"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ms2.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(ms2.EXPORTED)


def test_binding_structures_match_the_c_layout(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal what the C
    compiler lays out for include/ms2.h."""
    import subprocess
    probes = {
        "ms2_species": (ms2.Species, ["n_sites", "pos", "axis", "sigma", "mass", "inertia"]),
        "ms2_params": (ms2.Params, ["box", "coulomb_k", "elec", "precision"]),
        "ms2_system": (ms2.System, ["params", "n_mol", "n_steps", "dt", "rdf_rmax", "u0", "h_species",
                                    "h_omega"]),
        "ms2_samples": (ms2.Samples, ["steps_done", "sums", "moments", "h_rdf", "h_torque"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ms2.h"', "int main(void){"]
    for cname, (_, fields) in probes.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for _, (cls, fields) in probes.items():
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f in fields]
    assert got == want
