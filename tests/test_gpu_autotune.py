"""GPU: the autotuner picks a tiling by timing aqc_apply, the chosen plan is
still exact, and the choice is cached."""
import json

import numpy as np
import pytest

from oracle import sqh
from paper_1311_3938_amd import instances as I
from tests._gpu import to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu


def test_autotune_picks_and_caches(tmp_path):
    import torch
    from paper_1311_3938_amd import autotune, engine
    ctx = engine.Context(0)
    inst = I.workload_ec3_catalyst(n=17, m=13, n_pairs=17, T=5.0, seed=9)
    ham = engine.Hamiltonian(ctx, inst)
    path = str(tmp_path / "tune.json")
    best, ms, fresh = autotune.tune_cached(ctx, ham, inst, torch.complex64, path=path)
    assert fresh and ms > 0
    cache = json.load(open(path))
    assert list(cache.values())[0]["tiling"] == list(best)
    psi = I.random_state(17, np.random.default_rng(1))
    got = to_host(engine.apply(ctx, ham, 2.0, to_dev(psi, "c64")))
    assert rel_err(got, sqh.apply_h(inst, 2.0, psi)) < 5e-6
    ham2 = engine.Hamiltonian(ctx, inst)
    best2, _, fresh2 = autotune.tune_cached(ctx, ham2, inst, torch.complex64, path=path)
    assert not fresh2 and tuple(best2) == tuple(best)
    ham.free()
    ham2.free()
    ctx.close()


def test_set_tiling_rejects_bad_values():
    from paper_1311_3938_amd import _lib, engine
    import torch
    ctx = engine.Context(0)
    inst = I.workload_ec3_linear(n=10, m=8, T=2.0, seed=4)
    ham = engine.Hamiltonian(ctx, inst)
    with pytest.raises(_lib.AqcError):
        ham.set_tiling(torch.complex64, 15, 13, 4)
    with pytest.raises(_lib.AqcError):
        ham.set_tiling(torch.complex64, 13, 6, 6)
    with pytest.raises(_lib.AqcError):
        ham.set_tiling(torch.complex64, 13, 13, 4, 8)
    with pytest.raises(_lib.AqcError):
        ham.set_tiling(torch.complex64, 13, 13, 4, -1)
    ham.free()
    ctx.close()


def test_batch_autotune_picks_by_tick_time_and_caches(tmp_path):
    """Tuning by the tick time of a batch of replicas: the choice is one of the
    candidates, is applied (the tuned plan is still exact), and is cached
    under its own key beside the single-solve choice."""
    import torch
    from paper_1311_3938_amd import autotune, engine
    ctx = engine.Context(0)
    inst = I.workload_batch_member(3, n_lo=16, n_hi=16)
    ham = engine.Hamiltonian(ctx, inst)
    path = str(tmp_path / "tune.json")
    best, s_per_tick, fresh = autotune.tune_cached(ctx, ham, inst, torch.complex64, path=path, batch=True)
    assert fresh and s_per_tick > 0
    assert tuple(best) in [tuple(c) for c in autotune.BATCH_CANDIDATES[0]]
    key = list(json.load(open(path)).keys())[0]
    assert key.startswith("batch|")
    psi = I.random_state(16, np.random.default_rng(2))
    got = to_host(engine.apply(ctx, ham, 3.0, to_dev(psi, "c64")))
    assert rel_err(got, sqh.apply_h(inst, 3.0, psi)) < 5e-6
    ham2 = engine.Hamiltonian(ctx, inst)
    best2, _, fresh2 = autotune.tune_cached(ctx, ham2, inst, torch.complex64, path=path, batch=True)
    assert not fresh2 and tuple(best2) == tuple(best)
    ham.free()
    ham2.free()
    ctx.close()
