"""The C-ABI library loads and exports what include/nnplan.h declares; host-side validation
(no GPU needed: every case here is rejected before any HIP call)."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

from conftest import ROOT
from paper_1904_06680_amd import fleet, nnplan, proposal, scenes

HEADERS = [os.path.join(ROOT, "include", h) for h in ("nnplan.h", "nnproposal.h", "nnfleet.h")]


def declared_functions(header=None):
    names = set()
    for h in ([header] if header else HEADERS):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(nnp_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_surface():
    assert declared_functions(HEADERS[0]) == sorted(nnplan.EXPORTED)
    assert declared_functions(HEADERS[1]) == sorted(proposal.EXPORTED)
    assert declared_functions(HEADERS[2]) == sorted(fleet.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = nnplan.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert nnplan.nnp_version().startswith("nnplan")


def _c_layout(tmp_path, structs):
    """sizeof and offsetof of every field, as the C compiler lays out the header's structs."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nnfleet.h"',
             'int main(void){']
    for name, cls in structs:
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


def test_struct_layouts_match_header(tmp_path):
    structs = [("nnp_model", nnplan.nnp_model), ("nnp_problem", nnplan.nnp_problem),
               ("nnp_result", nnplan.nnp_result), ("nnp_rollout_out", nnplan.nnp_rollout_out),
               ("nnp_proposal_config", proposal.nnp_proposal_config),
               ("nnp_fleet_config", fleet.nnp_fleet_config),
               ("nnp_vehicle_spec", fleet.nnp_vehicle_spec),
               ("nnp_vehicle_state", fleet.nnp_vehicle_state)]
    lay = _c_layout(tmp_path, structs)
    for name, cls in structs:
        assert C.sizeof(cls) == lay[name], name
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == lay[f"{name}.{f}"], (name, f)


def _create(preset, **over):
    m = nnplan.make_model(preset)
    for k, v in over.items():
        if k == "widths":
            for i in range(4):
                m.widths[i] = v[i] if i < len(v) else 0
            m.n_layers = len(v) - 1
        else:
            setattr(m, k, v)
    return nnplan.nnp_create(m, 0)


@pytest.mark.parametrize("over, code", [
    (dict(dt=0.0), nnplan.NNP_EINVAL),
    (dict(dt=math.nan), nnplan.NNP_EINVAL),
    (dict(half_width=-1.0), nnplan.NNP_EINVAL),
    (dict(u_min=3.0, u_max=-3.0), nnplan.NNP_EINVAL),
    (dict(v_min=1.0, v_max=-1.0), nnplan.NNP_EINVAL),
    (dict(feature_set=nnplan.FEAT_SIX), nnplan.NNP_EINVAL),            # 8 inputs, 6 features
    (dict(widths=(8, 32, 32, 3)), nnplan.NNP_EINVAL),                  # 3 outputs
    (dict(widths=(8, 64, 2)), nnplan.NNP_EUNSUPPORTED),                # no compiled kernel
    (dict(lanes_per_sample=3), nnplan.NNP_EINVAL),
    (dict(lanes_per_sample=1), nnplan.NNP_EUNSUPPORTED),               # 1410 weights per lane
    (dict(block_threads=-256), nnplan.NNP_EINVAL),
    (dict(tile_pairs=3000), nnplan.NNP_EUNSUPPORTED),                  # no such launch shape
    (dict(lanes_per_sample=16, tile_pairs=4096), nnplan.NNP_EUNSUPPORTED),
    (dict(block_threads=128), nnplan.NNP_EUNSUPPORTED),
])
def test_invalid_models_are_rejected_before_device_work(over, code):
    rc, h = _create(scenes.C1, **over)
    assert rc == code and not h.value
    assert nnplan.nnp_last_error(None) != ""


def test_null_arguments():
    lib = nnplan.load_library()
    assert lib.nnp_create(None, None, 0) == nnplan.NNP_EINVAL
    h = C.c_void_p()
    assert lib.nnp_create(C.byref(h), None, 0) == nnplan.NNP_EINVAL
    assert lib.nnp_plan(None, None, None, None) == nnplan.NNP_EINVAL
    assert lib.nnp_rollout(None, None, None, None, None) == nnplan.NNP_EINVAL
    assert lib.nnp_sample_theta(0, 0, 0, 0, 10, None, None) == nnplan.NNP_EINVAL
    assert lib.nnp_n_theta(None) == nnplan.NNP_EINVAL
    assert lib.nnp_set_record_limit(None, 0) == nnplan.NNP_EINVAL
    assert lib.nnp_set_workspace_limit(None, 0) == nnplan.NNP_EINVAL
    lib.nnp_destroy(None)
