"""The C-ABI library: it loads, exports every entry point include/lif.h
declares, its structs have the layout the binding assumes, and host-side
validation rejects malformed input without touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1901_07993_amd import lif

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lif.h")

pytestmark = pytest.mark.skipif(not os.path.exists(lif.LIB_PATH), reason="liblif.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lif_[A-Za-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(lif.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", lif.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lif_\w+)", out))
    assert set(names) <= exported
    lib = lif.load()
    for n in names:
        assert hasattr(lib, n)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lif.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lif_blocks),'
                   ' sizeof(lif_opts), sizeof(lif_info), offsetof(lif_opts, stream), offsetof(lif_info, norms),'
                   ' offsetof(lif_blocks, on_device), offsetof(lif_opts, presize),'
                   ' offsetof(lif_info, iterations_redone), offsetof(lif_opts, refinement),'
                   ' offsetof(lif_info, cpl_products), offsetof(lif_opts, prec_switch),'
                   ' offsetof(lif_info, iterations_reduced), offsetof(lif_info, mem_reserved_bytes),'
                   ' offsetof(lif_opts, sym_delta), offsetof(lif_opts, residual_panel_rows),'
                   ' offsetof(lif_info, pair_panels), offsetof(lif_opts, update_panel_rows),'
                   ' offsetof(lif_info, leaf_gemm_launches_reduced), offsetof(lif_info, symbolic_launches),'
                   ' offsetof(lif_opts, update_prec), offsetof(lif_info, leaf_gemm_launches_fp32));'
                   ' return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(lif.Blocks), ctypes.sizeof(lif.Opts), ctypes.sizeof(lif.Info), lif.Opts.stream.offset,
            lif.Info.norms.offset, lif.Blocks.on_device.offset, lif.Opts.presize.offset,
            lif.Info.iterations_redone.offset, lif.Opts.refinement.offset, lif.Info.cpl_products.offset,
            lif.Opts.prec_switch.offset, lif.Info.iterations_reduced.offset, lif.Info.mem_reserved_bytes.offset,
            lif.Opts.sym_delta.offset, lif.Opts.residual_panel_rows.offset, lif.Info.pair_panels.offset,
            lif.Opts.update_panel_rows.offset, lif.Info.leaf_gemm_launches_reduced.offset,
            lif.Info.symbolic_launches.offset, lif.Opts.update_prec.offset, lif.Info.leaf_gemm_launches_fp32.offset]
    assert got == want


def test_default_options():
    o = lif.default_opts()
    assert (o.m, o.tau, o.prec, o.stop, o.max_iter, o.base_rows) == (4, 0.0, 0, 0, 100, 4096)
    assert o.tol == 1e-10 and o.timing == 0 and o.presize == 1 and o.refinement == 0 and o.prec_switch == 0.0
    assert o.sym_delta == 0 and o.residual_panel_rows == 0 and o.update_panel_rows == 0 and o.update_prec == 0


def _blocks(n, b, rows, cols, vals=None):
    nnzb = len(rows)
    v = np.zeros((nnzb, b, b)) if vals is None else vals
    return lif.HostBlocks(n, b, np.array(rows, np.int32), np.array(cols, np.int32), v)


@pytest.mark.parametrize("case,msg", [
    (dict(n=64, b=16, rows=[0], cols=[0]), "b must be 32 or 64"),
    (dict(n=128, b=64, rows=[1, 0], cols=[1, 0]), "not sorted"),
    (dict(n=128, b=64, rows=[0, 0], cols=[0, 0]), "not sorted"),
    (dict(n=128, b=64, rows=[0, 0, 1], cols=[0, 1, 1]), "not symmetric"),
    (dict(n=128, b=64, rows=[0, 2], cols=[0, 2]), "out of range"),
    (dict(n=0, b=64, rows=[], cols=[]), "n must be > 0"),
])
def test_invalid_inputs_rejected_on_host(case, msg):
    S = _blocks(**case)
    with pytest.raises(lif.LifError) as ei:
        lif.Factorization(S)
    assert ei.value.status == lif.ERR_INVALID and msg in str(ei.value)


def test_nonzero_padding_rejected():
    v = np.zeros((1, 64, 64))
    v[0, 63, 63] = 1.0
    S = _blocks(100, 64, [1], [1], None)
    S.vals = np.concatenate([v])
    with pytest.raises(lif.LifError) as ei:
        lif.Factorization(S)
    assert "beyond n" in str(ei.value)


@pytest.mark.parametrize("opt,val", [("m", 0), ("m", 9), ("tau", -1.0), ("prec", 7), ("stop", 3),
                                     ("max_iter", 0), ("base_rows", 16), ("start", 9),
                                     ("presize", 3), ("presize", -1), ("refinement", 2),
                                     ("refinement", -1), ("prec_switch", -1.0), ("prec_switch", float("nan")),
                                     ("sym_delta", 2), ("residual_panel_rows", -1), ("update_panel_rows", -1),
                                     ("timing", 3), ("update_prec", 2), ("update_prec", -1),
                                     # a reduced update needs the schedule (and a reduced prec)
                                     ("update_prec", 1)])
def test_invalid_options_rejected(opt, val):
    S = _blocks(64, 64, [0], [0], np.eye(64)[None])
    with pytest.raises(lif.LifError) as ei:
        lif.Factorization(S, **{opt: val})
    assert ei.value.status == lif.ERR_INVALID


def test_nonlocal_refinement_needs_fp64():
    S = _blocks(64, 64, [0], [0], np.eye(64)[None])
    with pytest.raises(lif.LifError) as ei:
        lif.Factorization(S, refinement=lif.REFINE_NONLOCAL, prec=lif.MIXED_BF16)
    assert ei.value.status == lif.ERR_INVALID and "needs prec" in str(ei.value)


@pytest.mark.parametrize("extra", [dict(prec=0, prec_switch=1e-2), dict(prec=2, prec_switch=0.0),
                                   dict(prec=2, prec_switch=1e-2, checkpoint=1)])
def test_reduced_update_needs_schedule_without_checkpoints(extra):
    S = _blocks(64, 64, [0], [0], np.eye(64)[None])
    with pytest.raises(lif.LifError) as ei:
        lif.Factorization(S, update_prec=lif.MIXED_FP32, **extra)
    assert ei.value.status == lif.ERR_INVALID and "update_prec" in str(ei.value)
