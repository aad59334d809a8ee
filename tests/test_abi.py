"""The C ABI library loads and exports every function include/maxflow.h
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2004_11227_amd", "libmaxflow.so")


def declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:maxflow|mf_pool)_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libmaxflow.so not built")
    lib = ctypes.CDLL(LIB)
    names = declared("maxflow.h")
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2004_11227_amd import maxflow as mfx
    assert set(declared("maxflow.h")) <= set(mfx.EXPORTS)


def test_workspace_bytes_and_validation_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libmaxflow.so not built")
    from paper_2004_11227_amd import maxflow as mfx
    p = mfx.make_params((2048, 2048), model="two", method="eb")
    n = mfx.workspace_bytes(p)
    plane = (2048 * 2048 + 2176) * 4     # 2-D planes are padded by 2176 elements
    # ctrl + 2 caps + 2 states of (u, qx, qy, ps, pt) planes
    assert 12 * plane <= n <= 12 * plane + 64 * 1024
    pb = mfx.make_params((2048, 2048), model="two", method="eb", storage="bf16")
    assert mfx.workspace_bytes(pb) < n
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), alpha=-1.0))
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), model="potts", nlabels=6))
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), method="eb", relax=2.0))


@pytest.mark.parametrize("shape", [(2048, 2048), (77, 131), (1, 5)])
def test_workspace_layout_reserves_every_region(shape):
    """The workspace covers every region a solver writes: ping-pong state
    buffers for the fused passes, the resolvent outputs and the scratch
    planes of rPDRQ (initialisation writes the resolvent outputs' u slot
    into the scratch planes, also for the fused pass that keeps b in LDS)."""
    if not os.path.exists(LIB):
        pytest.skip("libmaxflow.so not built")
    from paper_2004_11227_amd import maxflow as mfx

    def ws(**kw):
        return mfx.workspace_bytes(mfx.make_params(shape, model="two", **kw))

    H, W = shape
    pitch = (W + 3) // 4 * 4
    P = (pitch * H + 127) // 128 * 128 + 2176   # plane of the padded layout (elements; 2-D pad)
    Pd = (W * H + 127) // 128 * 128 + 2176       # plane of the dense layout

    def al(b):
        return (b + 255) // 256 * 256

    state_pad = al(4 * P) + al(8 * P) + al(4 * P) + al(4 * P)
    state_dense = al(4 * Pd) + al(8 * Pd) + al(4 * Pd) + al(4 * Pd)
    # fused rPDRQ: two state buffers + resolvent outputs + one FP32 scratch plane
    assert ws(method="dr", variant="fused") - ws(method="eb", variant="fused") == state_pad + al(4 * P)
    # in-place rPDRQ: one state buffer + resolvent outputs + scratch = the unfused rpADMM layout
    assert ws(method="dr", variant="unfused") == ws(method="eb", variant="unfused")
    # unfused rpADMM: dense planes, two state buffers and one FP32 scratch plane
    assert ws(method="eb", variant="unfused") - ws(method="eb", variant="fused") == \
        (al(8 * Pd) - al(8 * P)) + 2 * (state_dense - state_pad) + al(4 * Pd)


@pytest.mark.parametrize("shape", [(256, 256, 256), (40, 48, 70)])
def test_workspace_layout_3d(shape):
    """3-D fused two-label workspace: control block, 2 capacity planes and
    two state buffers of (u, q_x, q_y, q_z, p_s, p_t), each plane padded to
    128 elements plus 128 (the 3-D plane pad), rows to 4 elements."""
    if not os.path.exists(LIB):
        pytest.skip("libmaxflow.so not built")
    from paper_2004_11227_amd import maxflow as mfx
    D, H, W = shape
    pitch = (W + 3) // 4 * 4
    P = (pitch * H * D + 127) // 128 * 128 + 128

    def al(b):
        return (b + 255) // 256 * 256

    state = al(4 * P) + al(12 * P) + al(4 * P) + al(4 * P)
    caps = al(8 * P)
    n = mfx.workspace_bytes(mfx.make_params(shape, model="two", method="eb"))
    assert 0 <= n - (caps + 2 * state) <= 64 * 1024      # the control block
    bf = mfx.workspace_bytes(mfx.make_params(shape, model="two", method="eb", storage="bf16"))
    state_bf = al(4 * P) + al(6 * P) + al(2 * P) + al(2 * P)
    assert bf - (al(4 * P) + 2 * state_bf) == n - (caps + 2 * state)


@pytest.mark.parametrize("bad", [dict(method="eb", gs_sweeps=2), dict(method="dr", gs_sweeps=65),
                                 dict(method="fg", relax0=0.5, relax_ramp=5),
                                 dict(method="eb", relax=1.5, relax0=1.6, relax_ramp=5),
                                 dict(method="eb", relax0=0.5, relax_ramp=0)])
def test_invalid_preconditioner_variants_rejected(bad):
    from paper_2004_11227_amd import maxflow as mfx
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), **bad))


def test_valid_preconditioner_variants_accepted():
    from paper_2004_11227_amd import maxflow as mfx
    for kw in (dict(method="dr", gs_sweeps=4), dict(method="eb", relax=1.9, relax0=0.5, relax_ramp=10),
               dict(method="eb", relax0=1.9, relax_ramp=1)):
        assert mfx.workspace_bytes(mfx.make_params((16, 16), **kw)) > 0


def test_pdrq_layout_follows_the_sweep_count():
    """The fused rPDRQ pass (1 to 4 sweeps) keeps two state buffers with rows
    padded to a multiple of 4; the in-place launches (M_n with n > 4, or the
    unfused variant) keep one dense state, so their workspace is smaller
    (two-label and Potts)."""
    from paper_2004_11227_amd import maxflow as mfx
    for kw, top in ((dict(model="two"), 4), (dict(model="potts", nlabels=3), 3), (dict(model="potts", nlabels=8), 3)):
        ws = {n: mfx.workspace_bytes(mfx.make_params((64, 1001), method="dr", gs_sweeps=n, **kw))
              for n in (1, 2, top, top + 1, 64)}
        unf = mfx.workspace_bytes(mfx.make_params((64, 1001), method="dr", variant="unfused", **kw))
        assert ws[1] == ws[2] == ws[top]
        assert ws[top + 1] == ws[64] == unf < ws[1]


def test_image_capacities_validation_and_workspace():
    """cap_source="image" keeps one image plane instead of 2 or n capacity
    planes; bad powers, sources and non-finite levels are rejected, and the
    pool takes capacity planes only."""
    from paper_2004_11227_amd import maxflow as mfx
    for model, n in (("two", 2), ("potts", 8)):
        planes = mfx.workspace_bytes(mfx.make_params((256, 256), model=model, nlabels=n))
        image = mfx.workspace_bytes(mfx.make_params((256, 256), model=model, nlabels=n, cap_source="image",
                                                    levels=[0.1 * i for i in range(n)]))
        assert planes - image == (n - 1) * (256 * 256 + 2176) * 4     # padded 2-D planes
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), cap_source="image", cap_power=3, levels=[0.2, 0.8]))
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(mfx.make_params((16, 16), cap_source="image", levels=[float("nan"), 0.8]))
    p = mfx.make_params((16, 16))
    p.cap_source = 2
    with pytest.raises(mfx.MaxflowError):
        mfx.workspace_bytes(p)
    with pytest.raises(ValueError):
        mfx.make_params((16, 16), cap_source="image", levels=[0.0] * 9)
    assert mfx.lib().mf_pool_footprint(ctypes.byref(mfx.make_params((64, 64), cap_source="image",
                                                                     levels=[0.2, 0.8]))) == 0
