"""Launch graphs (FV_GRAPH) and the FFT launch-shape autotuner (FV_AUTOTUNE)."""
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("eps,tol", [(1e-6, 1e-6), (1e-10, 1e-12)])
def test_graph_replays_match_eager_and_oracle(gpu_lib, eps, tol):
    fv = gpu_lib
    p = synth.small_problem(70, n_ant=30, n_src=800, n_freq=4, hex_layout=True)
    other = synth.small_problem(71, n_ant=11, n_src=150, n_freq=2)
    with fv.Context(0) as c:
        # the type-3 launch sequence (a hex array would take the lattice path)
        hp = fv.HostProblem.of(p, eps=eps, flags=fv.NO_LATTICE)
        eager = c.simulate_problem(hp)
        ref = oracle.direct_problem(p)
        assert oracle.rel_l2(eager, ref) <= eps
        for r in range(4):
            g = c.simulate_problem(fv.HostProblem.of(p, eps=eps, flags=fv.GRAPH | fv.NO_LATTICE))
            assert oracle.rel_l2(g, eager) <= tol, r
            assert oracle.rel_l2(g, ref) <= eps, r
            # eager work of another shape between the replays
            c.simulate_problem(fv.HostProblem.of(other, eps=1e-6))
        # same sizes, new strengths: the replay must read the new inputs
        flux2 = p.flux * np.linspace(0.5, 1.5, p.n_src)[None, :]
        hp2 = fv.HostProblem(p.ant_enu, p.src_lmn, p.freq_hz, flux2, p.beam, eps, fv.GRAPH | fv.NO_LATTICE)
        g2 = c.simulate_problem(hp2)
        e2 = c.simulate_problem(fv.HostProblem(p.ant_enu, p.src_lmn, p.freq_hz, flux2, p.beam, eps, fv.NO_LATTICE))
        assert oracle.rel_l2(g2, e2) <= tol
        assert oracle.rel_l2(g2, eager) > 10 * tol


def test_autotune_persists_and_reuses(gpu_lib, tmp_path):
    fv = gpu_lib
    p = synth.small_problem(72, n_ant=40, n_src=1000, n_freq=3, hex_layout=True)
    path = tmp_path / "tune.json"
    ref = oracle.direct_problem(p)
    with fv.Context(0) as c:
        c.set_tune_cache(str(path))
        tune = fv.AUTOTUNE | fv.NO_LATTICE  # the FFT launch shape belongs to the type-3 path
        v1 = c.simulate_problem(fv.HostProblem.of(p, flags=tune))
        t1 = c.last_report["t_total_ms"]
        assert oracle.rel_l2(v1, ref) <= p.eps
        d = json.loads(path.read_text())
        assert len(d) == 1
        (key, ent), = d.items()
        assert key.startswith("d2_p32_") and ent["rows"] >= 1 and ent["lines"] >= 1 and ent["fft_ms"] > 0
        v2 = c.simulate_problem(fv.HostProblem.of(p, flags=tune))
        assert c.last_report["t_total_ms"] < t1
        assert oracle.rel_l2(v2, ref) <= p.eps
    with fv.Context(0) as c2:
        c2.set_tune_cache(str(path))
        v3 = c2.simulate_problem(fv.HostProblem.of(p, flags=tune))
        assert oracle.rel_l2(v3, ref) <= p.eps
        # a re-tune would rewrite the entry with a new measured time
        assert json.loads(path.read_text()) == d
