"""The docking entry point that allocates no device memory (exs_dock_batch_noalloc), through the
C ABI: its results equal those of exs_dock_batch + exs_get_best_poses bit for bit, on two calls
in a row (the second on a smaller input with other search settings, so the shared scratch
buffer holds the first call's contents), and a batch whose per-orientation results exceed the
buffer is refused before anything is launched."""
import sys

import numpy as np
import pytest

import exs_synth as S

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_11644_amd import binding
    binding.lib()
    return binding


def params(B, s, **kw):
    return B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                           s.clash_cutoff, s.clash_penalty, **kw)


def reference(B, bid, s, L, A):
    job = B.exs_dock_batch(bid, params(B, s))
    out = B.exs_get_best_poses(job, L, A)
    B.exs_release_job(job)
    return out


def no_alloc(B, torch, bid, s, batch):
    L, A, R = batch.n_ligands, int(batch.atom_offset[-1]), int(batch.rot_offset[-1])
    dev = torch.device("cuda")
    best = torch.full((L,), float("nan"), dtype=torch.float32, device=dev)
    orient = torch.full((L,), -1, dtype=torch.int32, device=dev)
    tau = torch.full((L,), -1, dtype=torch.int32, device=dev)
    theta = torch.full((max(R, 1),), 255, dtype=torch.uint8, device=dev)
    coords = torch.full((A, 3), float("nan"), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    B.exs_dock_batch_noalloc(bid, params(B, s), best, orient, tau, theta, coords, stream=stream)
    stream.synchronize()
    return dict(best=best.cpu().numpy(), orient=orient.cpu().numpy(), tau=tau.cpu().numpy(),
                theta=theta.cpu().numpy()[:R], coords=coords.cpu().numpy())


def assert_equal(batch, ref, got):
    L = batch.n_ligands
    assert np.array_equal(ref["best_score"], got["best"])
    assert np.array_equal(ref["desc"]["orient"], got["orient"])
    t = got["tau"].astype(np.uint32)
    tau = np.stack([(t >> (8 * a)) & 0xff for a in range(3)], axis=1).astype(np.uint8).view(np.int8)
    assert np.array_equal(ref["desc"]["tau"], tau)
    for l in range(L):
        r0, r1 = int(batch.rot_offset[l]), int(batch.rot_offset[l + 1])
        assert np.array_equal(ref["desc"]["theta"][l][:r1 - r0], got["theta"][r0:r1]), l
    assert np.array_equal(ref["coords"], got["coords"])


def test_no_alloc_equals_dock_batch_on_two_calls(B):
    import torch
    calls = [("scale", S.SCALE, 1500, S.SCALE.search), ("small", S.SMALL, 16, S.SearchSettings(100, 8, 2, 27))]
    for name, wl, n, s in calls:
        pocket = S.make_pocket(wl, 0)
        batch = S.make_ligand_batch(wl, 0, n)
        L, A = batch.n_ligands, int(batch.atom_offset[-1])
        log("no-alloc call: %s, %d ligands, K=%d S=%d P=%d T=%d" % (name, L, s.n_orient,
                                                                   s.torsion_steps, s.passes,
                                                                   s.n_offsets))
        pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
        try:
            bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
            try:
                got = no_alloc(B, torch, bid, s, batch)
                ref = reference(B, bid, s, L, A)
                assert_equal(batch, ref, got)
            finally:
                B.exs_release_ligands(bid)
        finally:
            B.exs_unload_pocket(pid)


def test_no_alloc_refuses_a_batch_beyond_its_buffer(B):
    import torch
    pocket = S.make_pocket("small")
    tri = S.Ligand(np.array([[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0]], np.float32),
                   np.array([0, 1, 2], np.uint8), np.array([[0, 1], [1, 2]], np.int32),
                   np.zeros(0, np.int32))
    batch = S.batch_from_ligands([tri] * 40000)          # 40,000 x 1,024 x 8 B > 256 MiB
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        try:
            dev = torch.device("cuda")
            out = [torch.zeros(40000, dtype=t, device=dev) for t in (torch.float32, torch.int32,
                                                                     torch.int32)]
            with pytest.raises(B.ExsError) as ei:
                B.exs_dock_batch_noalloc(bid, params(B, S.SearchSettings(1024, 8, 1, 1),
                                                     poses_per_lane=2), *out,
                                         None, torch.zeros((120000, 3), device=dev))
            assert ei.value.code == B.EXS_EINVAL and "split the batch" in str(ei.value)
            with pytest.raises(B.ExsError) as ei:           # ranking needs allocations
                B.exs_dock_batch_noalloc(bid, params(B, S.SearchSettings(8, 8, 1, 1), rank_keep=2),
                                         *out, None, torch.zeros((120000, 3), device=dev))
            assert ei.value.code == B.EXS_EINVAL
        finally:
            B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)
