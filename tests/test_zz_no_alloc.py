"""act_lem_decompose_noalloc through the C ABI: the no-allocation variant of
the hierarchical search (workspace in the library's fixed device array)
against act_lem_decompose (workspace allocated in the plan), on two calls in
a row, the second smaller, and its host-side size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2607_16629_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_16629_amd import act
    act.load()


def _cfg(samples):
    return W.paper_lem_config(samples=samples)


def test_lem_noalloc_matches_allocating_call_twice():
    """Two no-allocation calls in a row (19 windows x order 4 with 256 LHS
    samples, then 5 windows x order 3 with 64 samples, which reuses a smaller
    part of the same array) equal the allocating entry point bit for bit:
    parameters, coefficients, energies, flags, residuals and approximations."""
    from paper_2607_16629_amd import act
    wl = W.lem_eeg()
    g = wl.grid
    B = wl.signals.shape[0]
    plan = act.Plan(g, dict_="synth", prec="f64", max_batch=B, refine_steps=wl.refine_steps)
    calls = [(B, 4, 256, 71), (5, 3, 64, 72)]
    refs = []
    for nb, order, samples, seed in calls:
        lhs = W.lem_lhs(seed, nb, order, samples)
        refs.append(plan.lem_decompose(wl.signals[:nb], lhs, _cfg(samples), order))
    torch.cuda.synchronize()
    outs = []
    for nb, order, samples, seed in calls:
        lhs = torch.from_numpy(W.lem_lhs(seed, nb, order, samples)).cuda()
        resid = torch.from_numpy(wl.signals[:nb].copy()).cuda()
        out = plan.alloc_outputs(nb, order)
        plan.act_lem_decompose_noalloc(resid, lhs, _cfg(samples), order, out)
        out["resid"] = resid
        outs.append(out)
    torch.cuda.synchronize()
    for (nb, order, _, _), ref, out in zip(calls, refs, outs):
        for k in ("theta", "coef", "energy", "flags", "resid", "approx"):
            a, b = out[k].cpu().numpy(), ref[k].cpu().numpy()
            assert a.shape == b.shape, k
            np.testing.assert_array_equal(a, b, err_msg=f"{nb} {order} {k}")
        E = out["energy"].cpu().numpy()
        assert np.all(np.diff(E, axis=1) <= 1e-12 * E[:, :1])
    plan.close()


def test_lem_noalloc_rejects_work_beyond_the_array():
    """batch x candidates x 41 bytes above the array's size is refused on the
    host with ACT_ERR_INVALID before any launch; the entry point then still
    works within the limit."""
    from paper_2607_16629_amd import act
    wl = W.lem_eeg(windows=2)
    g = wl.grid
    nb = 50
    sig = np.tile(wl.signals, (nb // 2, 1))
    plan = act.Plan(g, dict_="synth", prec="f64", max_batch=nb, refine_steps=0)
    cfg = W.LemConfig(8192, 0, 4, (0, 0, 0, 0), ((1.0 / 256, 1.0, 1.0, 0.5),))
    assert nb * 8192 * 41 > act.LEM_SCRATCH_BYTES
    lhs = torch.from_numpy(W.lem_lhs(73, nb, 1, cfg.samples)).cuda()
    resid = torch.from_numpy(sig).cuda()
    out = plan.alloc_outputs(nb, 1)
    with pytest.raises(act.ActError) as e:
        plan.act_lem_decompose_noalloc(resid, lhs, cfg, 1, out)
    assert e.value.status == act.ACT_ERR_INVALID
    small = W.LemConfig(64, 0, 4, (0, 0, 0, 0), ((1.0 / 256, 1.0, 1.0, 0.5),))
    lhs2 = torch.from_numpy(W.lem_lhs(74, nb, 1, 64)).cuda()
    plan.act_lem_decompose_noalloc(resid, lhs2, small, 1, out)
    ref = plan.lem_decompose(sig, lhs2.cpu().numpy(), small, 1)
    torch.cuda.synchronize()
    for k in ("theta", "coef", "energy"):
        np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy())
    plan.close()
