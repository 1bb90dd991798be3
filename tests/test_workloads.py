"""Sizes of the benchmark workloads (host logic; no arithmetic of the method)."""
import workloads as W
from oracle.problem import Problem, next_5smooth


def test_sizes():
    cases = {W.vacuum_1x1x05().name: (705, 5640, (40, 40)),
             W.lossy_8x8x2().name: (195585, 12517440, (625, 625)),
             W.layered_16x16x4().name: (784385, 100401280, (1250, 1250)),
             W.batched_layered_8x8x2().name: (195585, 12517440, (625, 625))}
    for name, (n_ap, u, box) in cases.items():
        prob = Problem.from_cavity(W.by_name(name).cavity)
        assert (prob.n_ap, prob.unknowns, prob.box) == (n_ap, u, box)


def test_layer_splits():
    assert W.layered_16x16x4().cavity.layer_nz == (32, 64, 32)
    assert W.batched_layered_8x8x2().cavity.layer_nz == (16, 32, 16)
    assert len(W.batched_layered_8x8x2().incidences) == 128


def test_served_stream_reproducible():
    a = W.served_stream(50)
    b = W.served_stream(50)
    assert [r.workload.cavity for r in a] == [r.workload.cavity for r in b]
    for r in a:
        cav = r.workload.cavity
        assert sum(cav.layer_nz) == cav.nz and min(cav.layer_nz) >= 1
        assert cav.nx in (64, 128, 256, 384)


def test_next_5smooth():
    assert [next_5smooth(n) for n in (1, 7, 39, 618, 1237, 928)] == [1, 8, 40, 625, 1250, 960]


def test_example3_readings_differ_only_in_the_step_assignment():
    """Both readings of Example 3's interval counts: 2000 + 1000 intervals of one step, or
    1000 + 2000 with each layer's own step (bottom 2 wavelengths, top 1)."""
    one = Problem.from_cavity(W.example3_sweep().cavity)
    own = Problem.from_cavity(W.example3_sweep_steps().cavity)
    assert one.nz == own.nz == 3000 and one.c == own.c == 3.0
    assert one.layer_h == (1e-3, 1e-3)
    assert own.layer_h == (2.0 / 1000, 1.0 / 2000)
    assert own.h == 1.0 / 2000 and one.h == 1e-3       # aperture rows: the top layer's step
    assert one.layer_eps == own.layer_eps and (one.M, one.N) == (own.M, own.N) == (21, 21)
