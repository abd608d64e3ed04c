"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, and rejects bad geometry before any launch."""
import ctypes

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def P():
    import paper_2410_14900_amd as P
    return P


def test_library_exports_every_header_symbol(P):
    L = P._lib.lib()
    names = P.header_symbols()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(P._lib.SIGNATURES)


def test_struct_layout_matches_header():
    from paper_2410_14900_amd._lib import DcGrid, DcView
    assert ctypes.sizeof(DcView) == 15 * 8
    # int32 pairs pack, doubles align to 8
    assert DcGrid.du.offset == 8 and DcGrid.n_theta.offset == 24 and DcGrid.ds.offset == 32
    assert DcGrid.nx.offset == 40 and DcGrid.vx.offset == 56 and ctypes.sizeof(DcGrid) == 104


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3", "C5"])
def test_workload_geometries_validate(P, cfg):
    g, v = synth.config_geometry(cfg, n_views=12)
    assert P.validate(g, v) == (0, "")


def test_validate_rejects_bad_geometry(P):
    g, v = synth.config_geometry("C1", n_views=8)
    bad = v.subset(range(8))
    bad.src[2] += np.array([0.0, 0.0, 5.0])           # source off the detector normal
    st, msg = P.validate(g, bad)
    assert st == 1 and "normal" in msg
    bad = v.subset(range(8))
    bad.ex[1] *= 1.01                                  # not unit
    assert P.validate(g, bad)[0] == 1
    g2 = synth.Grid(**dict(g.as_dict(), vx=60.0))      # volume reaching behind the source
    st, msg = P.validate(g2, v)
    assert st == 1 and "front" in msg
    g3 = synth.Grid(**dict(g.as_dict(), nu=0))
    assert P.validate(g3, v)[0] == 2
    g4 = synth.Grid(**dict(g.as_dict(), du=-1.0))
    assert P.validate(g4, v)[0] == 1


def test_plan_create_without_device_fails_cleanly(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g, v = synth.config_geometry("C1", n_views=4)
    with pytest.raises(P.DcError):
        P.Plan(g, v)


@pytest.mark.parametrize("first, status", [
    ([1, 4, 8], "DC_ESHAPE"),      # does not start at 0
    ([0, 4, 7], "DC_ESHAPE"),      # does not end at n_views
    ([0, 4, 4, 8], "DC_ESHAPE"),   # an empty sample
    ([0, 6, 3, 8], "DC_ESHAPE"),   # not increasing
])
def test_batched_plan_rejects_bad_sample_lists_before_touching_the_device(P, first, status):
    g, v = synth.config_geometry("C1", n_views=8)
    with pytest.raises(P.DcError, match=status):
        P.Plan(g, v, first_view=first)


def test_batched_plan_rejects_more_samples_than_the_backprojection_grid_holds(P):
    import dataclasses
    g, v = synth.config_geometry("C1", n_views=8)
    g = dataclasses.replace(g, nz=1024, vz=0.03)          # 128 z-blocks of 8 slices
    first = list(range(0, 520)) + [520]                   # 520 one-view samples: 128 * 520 > 65535
    views = synth.sinusoid_orbit(520, 750.0, 1200.0)
    with pytest.raises(P.DcError, match="DC_ENOTSUP"):
        P.Plan(g, views, first_view=first)



def test_crofton_workspace_size_is_host_only():
    """The sample table holds 3 doubles per sinusoid sample (fine * count of them),
    plus 256 bytes of alignment slack; closed-form segments need none."""
    import synth
    from paper_2410_14900_amd import _lib, ops
    L = _lib.lib()
    sv = synth.sinusoid_orbit(24, 750.0, 1200.0)
    arr = ops.make_segments(sv.meta["segments"])
    assert L.dc_crofton_workspace_bytes(arr, 1, 64) == 3 * 64 * 24 * 8 + 256
    ca = synth.circle_arc_orbit(12, 36, 750.0, 1200.0, 30.0)
    assert L.dc_crofton_workspace_bytes(ops.make_segments(ca.meta["segments"]), 2, 64) == 256
    assert L.dc_crofton_workspace_bytes(arr, 0, 64) == 0
    assert L.dc_crofton_workspace_bytes(arr, 1, 0) == 0
