"""Training-level checks on the full configuration (sphere scene, 160^3
grids, 100^3 coarse mask, 8192 rays per batch drawn as the benchmark draws
them, targets from the scene generator):

* an all-ones segment mask leaves the sample list bit-identical to plain
  sampling (the proposal's fallback is the plain method);
* the fine stage trains: the photometric loss falls at least tenfold in
  1000 iterations (BF16 form);
* the learned proposal, trained online over those 1000 iterations (250
  updates on half batches), makes the
  fine pass evaluate fewer samples than an untrained proposal and than no
  proposal, and the render with its masks stays within 35 dB PSNR of the
  plain-sampled render of the same model (what the trained network gains
  over the method without it, at what cost in the image).
"""

import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
ITERS = 1000


@pytest.fixture(scope="module")
def setup(gpu_lib):
    import torch

    from paper_2111_11215_amd import api, experiment, train
    from paper_2111_11215_amd._lib import DVGO_BF16
    sp, cams, held, raw = synth.full_scene(0)
    n = synth.FULL_N
    voxel = 2.0 / (n - 1)
    step = 0.5 * voxel
    max_samples = int(math.ceil(2.0 * math.sqrt(3.0) / step)) + 1
    bmin, bmax = tuple(synth.BOX_MIN), tuple(synth.BOX_MAX)
    bits = api.coarse_mask_build(torch.as_tensor(raw).cuda(), bmin, bmax, api.coarse_raw_threshold(synth.FULL_TAU,
                                                                                                   step))
    coarse = (bits, bmin, bmax, raw.shape)
    spheres = torch.as_tensor(sp.as_f32_table()).cuda()
    batches = []
    for t in range(ITERS):
        rng = np.random.default_rng(1000 + t)
        o, d, *_ = synth.draw_pixels_with_replacement(rng, cams, 800, 800, 1000.0, 8192)
        jit = rng.random(8192).astype(np.float32)
        ot, dt = torch.as_tensor(o).cuda(), torch.as_tensor(d).cuda()
        batches.append(experiment.Batch(ot, dt, torch.as_tensor(jit).cuda(),
                                        api.scene_render(ot, dt, spheres, bmin, bmax, step / 4)))
    Ws, bs = synth.xavier_uniform_mlp(np.random.default_rng(7), (39, 128, 128, 3))
    flat = api.flat_from([Ws[0], bs[0], Ws[1], bs[1], Ws[2], bs[2]], api.MLP_SHAPES, "cuda:0")
    cfg = train.FineConfig(step=step, max_samples=max_samples, precision=DVGO_BF16, bf16_feat=True)
    model = train.FineModel(torch.zeros((n, n, n), device="cuda"), torch.zeros((n, n, n, 12), device="cuda"), flat,
                            bmin, bmax, api.low_density_bias(synth.FULL_ALPHA_INIT, voxel), cfg, coarse=coarse)

    def proposal():
        Wp, bp = synth.xavier_uniform_mlp(np.random.default_rng(11), (54, 64, 64, 32))
        return train.ProposalModel(api.flat_from([Wp[0], bp[0], Wp[1], bp[1], Wp[2], bp[2]], api.PROP_SHAPES,
                                                 "cuda:0"), bmin, bmax)
    views = []
    for c in held[:2]:
        o, d = synth.scenes.image_rays(c, 800, 800, 1000.0)
        views.append(experiment.View(torch.as_tensor(np.ascontiguousarray(o)).cuda(),
                                     torch.as_tensor(np.ascontiguousarray(d)).cuda(), None))
    return model, proposal, batches, views, coarse


def test_all_ones_mask_is_plain_sampling(setup):
    import torch

    model, _, batches, _, _ = setup
    b = batches[0]
    ones = torch.full((8192,), -1, dtype=torch.int32, device="cuda")
    s0 = model.sample(b.o, b.d, b.j)
    s1 = model.sample(b.o, b.d, b.j, seg_mask=ones)
    n = int(s0.n_kept.item())
    assert n == int(s1.n_kept.item()) > 0
    assert torch.equal(s0.ray_offset, s1.ray_offset)
    assert torch.equal(s0.sample_ray[:n], s1.sample_ray[:n]) and torch.equal(s0.sample_k[:n], s1.sample_k[:n])


def test_trained_proposal_gains_over_untrained_and_none(setup):
    from paper_2111_11215_amd import experiment
    model, proposal, batches, views, _ = setup
    prop = proposal()
    experiment.count_uniform(model, batches[:8])
    st = experiment.run(model, batches, ITERS, prop=prop, record_every=100)
    first, last = st.losses[0][1], st.losses[-1][1]
    probe = batches[-4:]
    none = experiment.evaluated_per_step(model, probe)
    untrained = experiment.evaluated_per_step(model, probe, proposal())
    trained = experiment.evaluated_per_step(model, probe, prop)
    psnr_tr = experiment.proposal_render_psnr(model, prop, views)
    print(f"  loss {first:.4f} -> {last:.5f}; evaluated samples per batch: none {none:.0f}, untrained "
          f"{untrained:.0f}, trained {trained:.0f}; masked render vs plain sampling {psnr_tr:.1f} dB; "
          f"all-segment rays at the end {st.fallback_rate[-1][1]:.3f}", flush=True)
    assert last < 0.1 * first
    assert untrained >= 0.99 * none
    assert trained <= 0.97 * none and trained < untrained
    assert psnr_tr >= 35.0
