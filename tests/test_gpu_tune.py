"""The autotuner: shape keys noted during a factorisation are measured on the
device, the table round-trips through JSON for this architecture, GEMM tile
entries leave every bit unchanged (all tiles sum each output's K terms in the
same order), and with the full table (which may pick other QR forms) results
still do not depend on the batch and stay within 10 eps of the oracle."""
import json

import numpy as np
import pytest

import workloads as W
from oracle import acr as OA

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _solve(acr, st, leaf, eps, b):
    import torch
    h = acr.acr_factor(_op(acr, st), leaf, eps, "fp64")
    x = acr.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    acr.acr_destroy(h)
    return x


def test_autotuner_table(gpu, tmp_path):
    import torch
    probs = [(W.varkappa(128), 32, 1e-8), (W.poisson(96, 40), 24, 1e-8), (W.convdiff(64), 16, 1e-9)]
    bs = [W.rhs(st.n, 3, seed=W.seed_for(3, 700 + i)) for i, (st, _, _) in enumerate(probs)]
    gpu.acr_tune_clear()
    ref = []
    gpu.acr_tune_record(True)
    for (st, leaf, eps), b in zip(probs, bs):
        ref.append(_solve(gpu, st, leaf, eps, b))
    gpu.acr_tune_record(False)
    added = gpu.acr_tune_run()
    print(f"tuned entries: {added}")
    assert added > 0
    path = tmp_path / "tune.json"
    gpu.acr_tune_save(path)
    table = json.loads(path.read_text())
    assert table["arch"].startswith("gfx950") and len(table["entries"]) == added
    kinds = {k.split(".")[0] for k in table["entries"]}
    print("kinds:", kinds, "sample:", list(table["entries"].items())[:6])
    # GEMM tiles only: the same bits as without a table
    gemm_only = dict(table, entries={k: v for k, v in table["entries"].items() if k.startswith("gemm.")})
    p2 = tmp_path / "gemm.json"
    p2.write_text(json.dumps(gemm_only))
    gpu.acr_tune_load(p2)
    for (st, leaf, eps), b, x0 in zip(probs, bs, ref):
        assert np.array_equal(_solve(gpu, st, leaf, eps, b), x0)
    # full table: batched equals solo, parity with the oracle
    gpu.acr_tune_load(path)
    ops = [_op(gpu, st) for st, _, _ in probs]
    for i, ((st, leaf, eps), b) in enumerate(zip(probs, bs)):
        # batched with another problem of the list (every side halves exactly to each leaf)
        hb = gpu.acr_factor_batched([ops[i], ops[(i + 1) % 3]], leaf, eps, "fp64")
        xb = gpu.acr_solve(hb[0], torch.from_numpy(b).cuda()).cpu().numpy()
        xs = _solve(gpu, st, leaf, eps, b)
        assert np.array_equal(xb, xs), f"problem {i}: batched differs from solo under the tuned table"
        xo = OA.solve(OA.factor(st, leaf, eps), st, b)
        assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 10 * eps
    # a table of another architecture is refused
    table["arch"] = "gfx000"
    p3 = tmp_path / "other.json"
    p3.write_text(json.dumps(table))
    with pytest.raises(gpu.ACRError) as ei:
        gpu.acr_tune_load(p3)
    assert ei.value.name == "ACR_ERR_INVALID_ARG"
    gpu.acr_tune_clear()


def test_mfma_tiles(gpu, tmp_path):
    """FP32 GEMM tiles on the matrix cores (kinds 10..14, picked only through the
    table): the five MFMA tiles give the same bits as each other, the results stay
    within the mixed-precision bound of the oracle, and the profiler shows the
    MFMA tiles ran."""
    import torch
    from bounds import mixed_forward_bound
    st, leaf, eps = W.varkappa(128), 32, 1e-8
    b = W.rhs(st.n, 2, seed=W.seed_for(3, 720))
    op = _op(gpu, st)

    def solve():
        h = gpu.acr_factor(op, leaf, eps, "mixed")
        x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
        gpu.acr_destroy(h)
        return x

    gpu.acr_tune_clear()
    gpu.acr_tune_record(True)
    x_vec = solve()
    gpu.acr_tune_record(False)
    gpu.acr_tune_run()
    path = tmp_path / "t.json"
    gpu.acr_tune_save(path)
    table = json.loads(path.read_text())
    keys = [k for k in table["entries"] if k.startswith("gemm.f.")]
    assert keys
    xo = OA.solve(OA.factor(st, leaf, eps), st, b)
    outs = []
    for kind in (10, 11, 12, 13, 14):
        t = dict(table, entries={k: kind for k in keys})
        p = tmp_path / f"k{kind}.json"
        p.write_text(json.dumps(t))
        gpu.acr_tune_load(p)
        gpu.acr_profile_start(None)
        outs.append(solve())
        paths = gpu.acr_profile_report().get("paths", {})
        gpu.acr_profile_start([])
        assert any(k.startswith("gemm.mfma") for k in paths), paths
    for x in outs[1:]:
        assert np.array_equal(x, outs[0])
    e_m = np.linalg.norm(outs[0] - xo) / np.linalg.norm(xo)
    e_v = np.linalg.norm(x_vec - xo) / np.linalg.norm(xo)
    print(f"mixed vs oracle: vector tiles {e_v:.2e}, MFMA tiles {e_m:.2e} (bound {mixed_forward_bound(eps):.1e}); "
          f"{len(keys)} FP32 GEMM keys, tuner picks {sorted(set(table['entries'][k] for k in keys))}")
    assert e_m <= mixed_forward_bound(eps) and e_v <= mixed_forward_bound(eps)
    gpu.acr_tune_clear()
