"""The allocation-free recording entry point (rdx_region_counts_static)
against the allocating one (rdx_region_counts) through the C ABI: per-region
sums of the same counts, bit for bit, on two calls in a row, the second on a
smaller simulation, and after windows that changed the counts."""
import sys

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
from tests.randmodels import random_counts, random_model

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_static_scratch_matches_allocating_entry_point():
    import torch
    from paper_1610_02258_amd import rdx

    rdx.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(97)
    S, R = 12, 10
    md = random_model(rng, S, R, 3)
    cases = [(I.box_mesh(30, 20, 20, 0.5e-6, jitter=0.1, seed=8), 3),   # 72,000 tets, 3 regions
             (I.box_mesh(3, 2, 2, 0.5e-6, seed=9), 3)]                   # 72 tets: fewer blocks
    for j, (mesh, n_regions) in enumerate(cases):
        mesh.region = rng.integers(0, n_regions, mesh.n_tets).astype(np.uint8)
        counts = random_counts(rng, S, mesh.n_tets, mean=2.0)
        big = counts.copy()
        big[0, :5] = (1 << 30) - 7  # sums past 2^32 (read only, never stepped)
        _say(f"case: static region sums, call {j}, T={mesh.n_tets} S={S} regions={n_regions}")
        sim = rdx.Sim(mesh.as_dict(), md, 50 + j)
        for w in range(2):
            if w == 0:
                sim.set_counts(big)
            else:
                sim.set_counts(counts)
                sim.step(3, stream=stream)
            got = torch.full((n_regions, S), -1, dtype=torch.int64, device=dev)
            ref = torch.full((n_regions, S), -2, dtype=torch.int64, device=dev)
            sim.region_counts_static(got, stream=stream)
            sim.region_counts(out=ref, stream=stream)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (j, w, got, ref)
            host = sim.get_counts().astype(np.int64)
            want = np.stack([host[:, mesh.region == g].sum(1) for g in range(n_regions)])
            assert np.array_equal(got.cpu().numpy(), want), (j, w)
        with pytest.raises(ValueError):
            sim.region_counts_static(torch.zeros((n_regions, S), dtype=torch.int32, device=dev))
        with pytest.raises(ValueError):
            sim.region_counts_static(torch.zeros((n_regions, S - 1), dtype=torch.int64, device=dev))
        sim.close()
