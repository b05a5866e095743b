"""The allocation-free sort (dust_bin_noalloc) against dust_bin: the same
permutation, bin starts and permuted particle arrays, bit for bit, on two
calls in a row (the second with fewer particles), in both key modes."""
import numpy as np
import pytest

from paper_1908_10793_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _particles(n, C, seed):
    r = np.random.default_rng(seed)
    cells = r.integers(-1, C, size=n).astype(np.int32)
    cells[r.random(n) < 0.03] = -1
    P = {"cell": torch.from_numpy(cells).cuda(),
         "off": [torch.from_numpy(r.random(n, dtype=np.float32) - 0.5).cuda() for _ in range(3)],
         "mom": [torch.from_numpy(r.standard_normal(n).astype(np.float32)).cuda() for _ in range(3)],
         "species": torch.from_numpy(r.integers(0, 4, size=n).astype(np.uint8)).cuda(),
         "id": torch.arange(n, dtype=torch.int32).cuda()}
    return P


def _clone(P):
    return {k: ([x.clone() for x in v] if isinstance(v, list) else v.clone()) for k, v in P.items()}


def _flat(P):
    out = []
    for k in sorted(P):
        v = P[k]
        out.extend(v if isinstance(v, list) else [v])
    return out


@pytest.mark.parametrize("mode", ["cell", "tile"])
def test_noalloc_sort_matches_dust_bin(mode):
    from paper_1908_10793_amd import dust
    w = synth.batched_boxes(sizes=(40, 24, 9), max_per_species=1)
    ctx = dust.context_for(w)
    ctx.set_tile(8, 4, 8, 0)
    _, C = ctx.grid_size()
    for call, (n, seed) in enumerate(((dust.BIN_NOALLOC_MAX - 3, 11), (70001, 12))):
        print(f"[no_alloc] mode={mode} call={call} n={n}", flush=True)
        P = _particles(n, C, seed)
        Q = _clone(P)
        perm_a = torch.empty(n, dtype=torch.int32, device="cuda")
        perm_b = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        start_a = torch.empty(C + 1, dtype=torch.int64, device="cuda")
        start_b = torch.full((C + 1,), -7, dtype=torch.int64, device="cuda")
        ctx.bin(P, key_mode=mode, perm=perm_a, bin_start=start_a, apply=True)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.bin_noalloc(Q, key_mode=mode, perm=perm_b, bin_start=start_b, apply=True)
        torch.cuda.synchronize()
        if call == 1:
            # the second call allocates nothing on the device
            assert torch.cuda.mem_get_info()[0] == free0
        assert torch.equal(perm_a, perm_b)
        assert torch.equal(start_a, start_b)
        for a, b in zip(_flat(P), _flat(Q)):
            assert torch.equal(a, b)
        # the permutation is the stable sort of the keys (ids follow it)
        assert torch.equal(Q["id"], perm_b)


def test_noalloc_sort_refuses_more_than_its_maximum():
    from paper_1908_10793_amd import dust
    w = synth.batched_boxes(sizes=(8,), max_per_species=1)
    ctx = dust.context_for(w)
    n = dust.BIN_NOALLOC_MAX + 1
    P = {"cell": torch.zeros(n, dtype=torch.int32, device="cuda"),
         "off": [torch.zeros(n, device="cuda") for _ in range(3)],
         "mom": [torch.zeros(n, device="cuda") for _ in range(3)]}
    with pytest.raises(dust.DustError, match="at most"):
        ctx.bin_noalloc(P, key_mode="cell", apply=True)
    assert torch.equal(P["cell"], torch.zeros(n, dtype=torch.int32, device="cuda"))


def test_noalloc_sort_of_no_particles():
    from paper_1908_10793_amd import dust
    w = synth.batched_boxes(sizes=(8,), max_per_species=1)
    ctx = dust.context_for(w)
    _, C = ctx.grid_size()
    P = {"cell": torch.zeros(0, dtype=torch.int32, device="cuda"),
         "off": [torch.zeros(0, device="cuda") for _ in range(3)],
         "mom": [torch.zeros(0, device="cuda") for _ in range(3)]}
    start = torch.full((C + 1,), 5, dtype=torch.int64, device="cuda")
    ctx.bin_noalloc(P, key_mode="tile", bin_start=start, apply=True)
    torch.cuda.synchronize()
    assert torch.equal(start, torch.zeros(C + 1, dtype=torch.int64, device="cuda"))
