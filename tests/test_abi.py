"""The C-ABI library loads and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libmrf.h")
LIB = os.path.join(ROOT, "paper_1506_05393_amd", "libmrf.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(mrf_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mrf_simulate_dictionary", "mrf_match_bruteforce", "mrf_context_create",
              "mrf_sequence_create", "mrf_grid_size", "mrf_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmrf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmrf.so not built")
def test_binding_declares_every_header_symbol():
    from paper_1506_05393_amd import _lib
    assert sorted(_lib.exported_names()) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmrf.so not built")
def test_host_only_calls_without_gpu():
    """Calls that touch no device: status strings and grid validation."""
    import numpy as np
    from paper_1506_05393_amd import _lib, api, inputs
    lib = _lib.load()
    assert lib.mrf_status_str(0) == b"ok"
    assert lib.mrf_version().startswith(b"libmrf")
    g = inputs.make_grid([100.0, 200.0, 300.0], [10.0, 20.0], [-4.0, 0.0, 4.0, 8.0])
    assert lib.mrf_grid_size(api.GridArg(g).ptr) == 24
    g4 = inputs.make_grid([100.0], [10.0], [0.0], [0.9, 1.0, 1.1])
    assert lib.mrf_grid_size(api.GridArg(g4).ptr) == 3
    bad = inputs.Grid(np.array([200.0, 100.0]), np.array([10.0]), np.array([0.0]))
    assert lib.mrf_grid_size(api.GridArg(bad).ptr) == -1
    assert b"strictly increasing" in lib.mrf_last_error()
    neg = inputs.Grid(np.array([-1.0]), np.array([10.0]), np.array([0.0]))
    assert lib.mrf_grid_size(api.GridArg(neg).ptr) == -1
    # argument checks of the peak probes come before any device work
    assert lib.mrf_probe_mfma(None, 0, 10, None, 256, None, None) == 1  # MRF_ERR_INVALID
    assert lib.mrf_probe_mfma_varied(None, 10, None, 256, None, None) == 1
    assert lib.mrf_probe_write(None, None, 16, 0, None) == 1  # MRF_ERR_INVALID


def test_local_refine_schedule_builder():
    """mrf_zoom_schedule_local (host only): unit 2-D (T1, T2) zoom, unit df zoom
    (and unit B1 zoom with a B1 axis), the same list repeated as the outer loop."""
    from paper_1506_05393_amd import api
    from paper_1506_05393_amd import inputs as I
    g = I.make_grid([300.0, 700.0, 1200.0], [30.0, 60.0], [-4.0, 0.0, 4.0])
    s = api.schedule_local(g, outer_max=5)
    kinds = [(x["kind"], x["axis0"], x["step0"]) for x in s["stages"]]
    assert kinds == [(4, 0, 1), (3, 2, 1)] and s["stages"][0]["axis1"] == 1
    assert s["outer"] == s["stages"] and s["outer_max"] == 5
    g4 = I.make_grid([300.0, 700.0], [30.0, 60.0], [0.0], [0.9, 1.0, 1.1])
    s4 = api.schedule_local(g4)
    assert [(x["kind"], x["axis0"]) for x in s4["stages"]] == [(4, 0), (3, 2), (3, 3)]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmrf.so not built")
def test_prior_schedule_builder_matches_hand_worked_and_oracle(orc):
    """mrf_zoom_schedule_prior (host only) gives the neighbour-prior half
    widths of Experiment 3 worked by hand in the oracle pins, and the oracle's
    conversion on random grids."""
    import numpy as np
    from paper_1506_05393_amd import api, workloads
    from paper_1506_05393_amd import inputs as I
    assert api.prior_half_widths(workloads.slice64().grid) == [300, 160, 150, -1]
    assert api.prior_half_widths(workloads.volume(1, 8).grid) == [3000, 800, 300, 60]
    assert api.prior_half_widths(workloads.small_dgs().grid) == [93, 82, 38, -1]
    g = I.make_grid([100.0, 160.0, 220.0], [10.0, 20.0], [-60.0, 0.0, 60.0])
    assert api.prior_half_widths(g, 150.0, 25.0, 150.0) == [3, 3, 3, -1]
    rng = np.random.default_rng(8)
    for _ in range(40):
        ax = [np.cumsum(rng.uniform(0.5, 30.0, int(rng.integers(1, 12)))) for _ in range(3)]
        b1 = np.cumsum(rng.uniform(0.001, 0.05, int(rng.integers(0, 6))))
        g = I.make_grid(ax[0], ax[1], ax[2] - 50.0, b1 if len(b1) else None)
        half = list(rng.uniform(-5.0, 400.0, 3)) + [float(rng.uniform(0.0, 0.3))]
        assert api.prior_half_widths(g, *half) == orc.prior_half(g, half)
    s = api.schedule_with_prior(dict(stages=[], starts=[[0, 0, 0, 0]]), workloads.slice64().grid)
    assert s["prior_half"] == [300, 160, 150, -1]


def test_finest_objective_builder_matches_oracle(orc):
    """mrf_zoom_schedule_finest_objective (host only) flags the same stages
    as the oracle's builder: the unit-step ones of both lists."""
    from paper_1506_05393_amd import api, workloads
    for w in (workloads.small_dgs(), workloads.slice64(), workloads.volume(1, 8)):
        s = orc.schedule_paper(w.seq, w.grid)
        a = api.schedule_finest_objective(s, 1)
        b = orc.schedule_finest_objective(s, 1)
        assert a == b
        for st in a["stages"] + a["outer"]:
            unit = (st["kind"] == 4 and st["step0"] <= 1 and st["step1"] <= 1) or \
                   (st["kind"] in (0, 1, 3) and st["step0"] <= 1)
            assert st["objective"] == (1 if unit else 0)
        assert api.schedule_finest_objective(a, 0) == s
