"""GPU tests of the large-problem memory policies, driven on small inputs by
a memory cap (opts.mem_cap_bytes sizes the policies when it is below the
GPU's memory):

* iterations on one stream with every buffer freed after its last reader;
* products written as kept blocks only, in chunks, each chunk's store cut to
  its kept blocks (the untruncated product is never held), their pair lists
  built one panel of block rows at a time;
* the true residual formed by panels of block columns.

None of them changes a value: a capped factorization gives Z bit for bit
and the same iteration counts as an uncapped one (FP64, symmetric delta
update, and the BF16 precision schedule, whose input copies are then made
from the stored blocks instead of by the producing product).  The residual
by panels forms every block of I - Z^T S Z as the whole product does; only
the order of the final sum of squares differs (1e-12 relative bound).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import blocks_to_dense, config_matrix, overlap_blocks, water_cluster  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(S, cap, **opts):
    with lif.Factorization(dev(S), mem_cap_bytes=cap, **opts) as f:
        info = f.localized()
        Z = f.get_Z()
        res = f.residual()
    return info, Z, res


@pytest.mark.parametrize("variant", ["fp64", "fp64_sym", "bf16_schedule_sym", "chain_fp64",
                                     "bf16_schedule_sym_f32update"])
def test_capped_run_matches_uncapped(variant):
    if variant.startswith("chain"):
        # several problems per level, sparse products (a few block products
        # per output block), some problems stopping before others
        S, cfg = config_matrix(1, count=150)       # n = 3000, b = 64, 47 block rows
        opts = dict(tau=cfg["tau"], base_rows=512)
    else:
        c_, e_ = water_cluster(300, 17)
        S = overlap_blocks(c_, e_, 32)             # n = 2100, b = 32, 66 block rows
        opts = dict(tau=1e-6, base_rows=512)
    if "sym" in variant:
        opts["sym_delta"] = 1
    if "bf16" in variant:
        opts.update(prec=lif.MIXED_BF16, prec_switch=1e-2)
    if "f32update" in variant:
        opts["update_prec"] = lif.MIXED_FP32
    say(f"case memory cap water-300 n={S.n} {variant}")
    i0, Z0, r0 = _run(S, 0, **opts)
    peak = int(i0["mem_peak_bytes"])
    # a quarter above the uncapped peak (the capped runs need about 0.7 of
    # it): every policy switches on (one stream once an iteration's buffers
    # exceed a quarter of the cap or take the pool past half of it,
    # compaction above 1/64 of it, chunks of 1/16, pair lists in row panels
    # above 1/512, residual panels of 1/16)
    cap = peak + peak // 4
    if variant == "fp64":
        # three quarters of the uncapped peak (sums sized exactly keep the
        # capped run near 0.6 of it): the pool then holds more than half of
        # the cap when the largest products list their pairs, which are built
        # by row panels
        cap = 3 * peak // 4
    i1, Z1, r1 = _run(S, cap, **opts)
    say(f"  uncapped peak {peak / 2**20:.1f} MiB, capped peak {i1['mem_peak_bytes'] / 2**20:.1f} MiB; "
        f"iterations {i0['iterations_total']} / {i1['iterations_total']}; residual {r0:.6e} / {r1:.6e}; "
        f"compacted {i0['products_compacted']} / {i1['products_compacted']}, "
        f"pair panels {i0['pair_panels']} / {i1['pair_panels']}")
    assert i0["products_compacted"] == 0 and i0["pair_panels"] == 0
    assert i1["products_compacted"] > 0
    if variant == "fp64":  # the full products' pair lists exceed the panel budget
        assert i1["pair_panels"] > 0
    zblk = Z0.vals.shape[1] * Z0.vals.shape[2] * 8
    assert Z0.nnzb * zblk > cap / 64, "the factor is too small for the cap to compact its products"
    assert i1["mem_peak_bytes"] <= cap
    assert i0["iterations_total"] == i1["iterations_total"]
    assert i0["iterations_reduced"] == i1["iterations_reduced"]
    assert np.array_equal(Z0.brow, Z1.brow) and np.array_equal(Z0.bcol, Z1.bcol)
    assert np.array_equal(Z0.vals, Z1.vals)
    assert abs(r0 - r1) <= 1e-12 * r0


@pytest.mark.parametrize("rows", [1, 5, 21, 66])
def test_residual_by_panels(rows):
    c_, e_ = water_cluster(300, 17)
    S = overlap_blocks(c_, e_, 32)                 # 66 block rows: panels of 1, 5 (ragged), 21, all
    say(f"case residual panels of {rows} block columns")
    with lif.Factorization(dev(S), tau=1e-6, base_rows=512) as f:
        f.localized()
        whole = f.residual()
    with lif.Factorization(dev(S), tau=1e-6, base_rows=512, residual_panel_rows=rows) as f:
        f.localized()
        panels = f.residual()
    say(f"  whole {whole:.15e} panels {panels:.15e}")
    assert abs(whole - panels) <= 1e-12 * whole


def test_residual_by_panels_irsi_exact():
    # tau = 0: Z converged to the rounding floor; panels reproduce the value
    S, _ = config_matrix(0)
    lam = float(np.linalg.eigvalsh(blocks_to_dense(S))[-1])
    say("case residual panels water-100 irsi")
    with lif.Factorization(dev(S), start=lif.START_INV_SQRT_LMAX, start_value=lam) as f:
        f.refine()
        whole = f.residual()
    with lif.Factorization(dev(S), start=lif.START_INV_SQRT_LMAX, start_value=lam, residual_panel_rows=4) as f:
        f.refine()
        panels = f.residual()
    assert whole < 1e-12 and abs(whole - panels) <= 1e-12 * whole


@pytest.mark.parametrize("variant,rows", [("fp64", 1), ("fp64", 7), ("fp64_sym", 5), ("bf16_schedule_sym", 13),
                                          ("irsi_fp64", 9), ("chain_fp64", 4),
                                          ("bf16_schedule_sym_f32update", 13), ("chain_bf16_schedule_f32update", 4)])
def test_delta_update_by_panels_matches_whole(variant, rows):
    # the delta update formed `rows` block rows at a time (neither product
    # held whole) gives the same factor bit for bit
    if variant.startswith("chain"):
        S, cfg = config_matrix(1, count=150)       # n = 3000, b = 64, 47 block rows
        opts = dict(tau=cfg["tau"], base_rows=512)
    else:
        c_, e_ = water_cluster(300, 17)
        S = overlap_blocks(c_, e_, 32)             # n = 2100, b = 32, 66 block rows
        opts = dict(tau=1e-6, base_rows=512)
    if "sym" in variant:
        opts["sym_delta"] = 1
    if "bf16" in variant:
        opts.update(prec=lif.MIXED_BF16, prec_switch=1e-2)
    if "f32update" in variant:
        opts["update_prec"] = lif.MIXED_FP32
    say(f"case delta update by panels of {rows} block rows, {variant}, n={S.n}")

    def run(**extra):
        with lif.Factorization(dev(S), **opts, **extra) as f:
            info = f.refine() if variant.startswith("irsi") else f.localized()
            return info, f.get_Z()

    i0, Z0 = run()
    i1, Z1 = run(update_panel_rows=rows)
    say(f"  iterations {i0['iterations_total']} / {i1['iterations_total']}, peak "
        f"{i0['mem_peak_bytes'] / 2**20:.1f} / {i1['mem_peak_bytes'] / 2**20:.1f} MiB")
    assert i0["iterations_total"] == i1["iterations_total"]
    assert i0["norms"] == i1["norms"]
    assert np.array_equal(Z0.brow, Z1.brow) and np.array_equal(Z0.bcol, Z1.bcol)
    assert np.array_equal(Z0.vals, Z1.vals)
