"""The library's calls run on the stream they are given (the binding passes torch's current
stream): two contexts stepped on two side streams at once give the bits of sequential runs on
the default stream; and an even number of steps captured into a HIP graph replays to the bits
of the same steps run eagerly, replay after replay, with eager work between the replays."""
import numpy as np
import pytest

import synth
from tests._common import needs_gpu, spec_params

pytestmark = [pytest.mark.gpu, needs_gpu]

LES = dict(tau=0.6, visc="smagorinsky", drive="yu", nu0=0.1 / 3.0, c_smag=0.2)


def _sim(shape, seed):
    import torch
    from paper_1704_07559_amd import lbm
    _, cp, _ = spec_params(shape, **LES)
    sim = lbm.LBM(cp)
    g0 = synth.random_state(19, shape, seed=seed, scale=3e-3).astype(np.float32)
    sim.set_populations(torch.as_tensor(g0).cuda())
    return sim


def test_two_contexts_on_two_streams():
    import torch
    from paper_1704_07559_amd import capi
    shape = (6, 40, 128)
    ref = []
    for seed in (1, 2):
        sim = _sim(shape, seed)
        S = torch.empty((6,) + shape, device="cuda")
        sim.step(10, S_out=S)
        torch.cuda.synchronize()
        ref.append((sim.populations(), S.clone(), sim.s_nu.clone()))
        sim.close()
    sims = [_sim(shape, 1), _sim(shape, 2)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty((6,) + shape, device="cuda") for _ in sims]
    for n in range(10):  # interleaved launches on the two streams
        for sim, st, S in zip(sims, streams, outs):
            with torch.cuda.stream(st):
                sim.step(1, S_out=S, strain_kind=capi.LBM_STRAIN_YU)
    torch.cuda.synchronize()
    for sim, S, (g, Sr, sr) in zip(sims, outs, ref):
        assert torch.equal(sim.populations(), g) and torch.equal(S, Sr) and torch.equal(sim.s_nu, sr)
        assert sim.step_count == 10
        sim.close()


def test_steps_captured_in_a_graph_replay_exactly():
    import torch
    shape = (4, 24, 64)
    eager, cap = _sim(shape, 3), _sim(shape, 3)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    S_cap = torch.empty((6,) + shape, device="cuda")
    # the library alternates its two population buffers on the host, so a graph holds an even
    # number of steps and every replay starts from the buffer the capture started from
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            cap.step(1, S_out=S_cap)
            cap.step(1, S_out=S_cap)
    torch.cuda.synchronize()
    S_eager = torch.empty_like(S_cap)
    for rep in range(4):
        graph.replay()
        eager.step(2, S_out=S_eager)
        torch.cuda.synchronize()
        assert torch.equal(cap.populations(), eager.populations()), rep
        assert torch.equal(S_cap, S_eager) and torch.equal(cap.s_nu, eager.s_nu), rep
        d = cap.reduce()                       # eager work between the replays
        assert d["nonfinite"] == 0
    eager.close()
    cap.close()
