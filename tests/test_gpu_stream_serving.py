"""Stateful stream serving on the sliding-window driver (serve.StreamServer)
through the C ABI: frames of 6 camera streams arriving faster than the steps
run, so several streams share most steps and the mix changes from step to
step.  Each stream's result (keyframes, edges, window poses and depths, whole
trajectory) must equal the same frames stepped alone in a driver of its own:
the decisions bit-exact, poses within 1e-6 m / 1e-4 deg and inverse depths
within 1e-6 relative (FP64).  The two runs differ only in how the solver
chunks the batch."""
import numpy as np
import pytest

from paper_2208_04726_amd import synth
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def test_streams_served_in_a_mix_equal_the_streams_alone():
    need_gpu()
    from paper_2208_04726_amd.serve import StreamServer, frame_latency_summary, frame_trace
    from paper_2208_04726_amd.vo import Driver
    S, F = 6, 30
    streams = [synth.make_stream(F + 2, 32, seed=[2208, 40, i]) for i in range(S)]
    reqs = frame_trace(S, F, fps=3000.0, seed=4)
    mix = Driver(streams, precision="fp64")
    res = StreamServer(mix).run(reqs)
    summ = frame_latency_summary(res)
    print("served:", summ, flush=True)
    assert sorted(res) == list(range(S * F))
    assert summ["mean_batch"] > 1.5
    n_mix, kf_mix, _, _ = mix.read()
    for s in range(S):
        alone = Driver([streams[s]], precision="fp64")
        for f in range(F):
            alone.step(np.array([f], np.int32))
        n1, kf1, _, _ = alone.read()
        k = int(n1[0])
        assert int(n_mix[s]) == k and kf_mix[s, :k].tolist() == kf1[0, :k].tolist(), s
        pm, dm, gm, fm = mix.window(s)
        p1, d1, g1, f1 = alone.window(0)
        assert gm.tolist() == g1.tolist() and fm.tolist() == f1.tolist(), s
        dc, dr = synth.pose_errors(pm[:k], p1[:k])
        dd = float(np.max(np.abs(dm[:k * 32] - d1[:k * 32]) / np.abs(d1[:k * 32])))
        tm, t1 = mix.trajectory(s), alone.trajectory(0)
        assert sorted(tm) == sorted(t1) == list(range(F))
        tc, tr = synth.pose_errors(np.stack([tm[f] for f in range(F)]), np.stack([t1[f] for f in range(F)]))
        print(f"stream {s}: window {dc:.1e} m {dr:.1e} deg depth {dd:.1e}; trajectory {tc:.1e} m {tr:.1e} deg")
        assert max(dc, tc) <= 1e-6 and max(dr, tr) <= 1e-4 and dd <= 1e-6
        alone.close()
    mix.close()
