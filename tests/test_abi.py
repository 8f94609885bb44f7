"""Host-side checks of the C ABI: the library loads, exports what the header
declares, and rejects invalid descriptors before touching any device."""
import ctypes
import os
import re

import pytest

from paper_1905_03277_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "hmfsr.h")).read()
    return sorted(set(re.findall(r"\b(hmfsr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    syms = header_symbols()
    assert syms, "no declarations found"
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in hmfsr.h but not exported"
    assert sorted(binding.EXPORTED) == syms


def test_version_and_strerror():
    assert binding.hmfsr_version() == 140
    assert "INVALID" in binding.strerror(binding.HMFSR_E_INVALID)
    assert "unknown" in binding.strerror(-99)


def _good():
    d = synth.Desc(4, 64, 96, tile_size=16, scale=1.5)
    return binding.make_desc(d), binding.make_tuning(synth.TUNING_SNR22)


def _call(desc, tun, ptr=1):
    # Invalid descriptors are rejected on the host, before any HIP call; the
    # dummy pointers are never dereferenced.
    return binding.lib().hmfsr_merge(ctypes.byref(desc), ctypes.byref(tun), ptr, ptr, ptr, None, None)


@pytest.mark.parametrize("field,value", [
    ("n_frames", 0), ("height", 63), ("width", 2), ("ref_frame", 4), ("ref_frame", -1),
    ("black_level", 5000.0), ("noise_b", 0.0), ("noise_a", -1e-3), ("tile_size", 15),
    ("tile_size", 0), ("tile_size", 6), ("scale", 0.5), ("scale", float("nan")), ("out_height", 95),
    ("out_width", 143),
])
def test_invalid_descriptor_rejected(field, value):
    desc, tun = _good()
    setattr(desc, field, value)
    assert _call(desc, tun) == binding.HMFSR_E_INVALID


@pytest.mark.parametrize("field,value", [
    ("k_detail", 0.0), ("k_denoise", -1.0), ("d_tr", 0.0), ("k_stretch", 0.0),
    ("k_shrink", float("inf")), ("t", float("nan")), ("s", -1.0), ("m_th", -0.1),
    ("hf_ratio", -0.1), ("hf_ratio", float("nan")),
])
def test_invalid_tuning_rejected(field, value):
    desc, tun = _good()
    setattr(tun, field, value)
    assert _call(desc, tun) == binding.HMFSR_E_INVALID


def test_unknown_cfa_unsupported():
    desc, tun = _good()
    desc.cfa = 7
    assert _call(desc, tun) == binding.HMFSR_E_UNSUPPORTED


def test_null_pointers_rejected():
    desc, tun = _good()
    assert _call(desc, tun, ptr=None) == binding.HMFSR_E_INVALID
    assert binding.lib().hmfsr_merge(None, ctypes.byref(tun), 1, 1, 1, None, None) == binding.HMFSR_E_INVALID


def test_binding_raises():
    desc, tun = _good()
    desc.n_frames = 0
    with pytest.raises(binding.HmfsrError):
        binding.hmfsr_merge(desc, tun, 1, 1, 1)


def _call_bwd(desc, tun, ptr=4, grad=4):
    return binding.lib().hmfsr_merge_backward(ctypes.byref(desc), ctypes.byref(tun), ptr, ptr, None,
                                              ptr, grad, grad, None)


@pytest.mark.parametrize("field,value", [("n_frames", 0), ("scale", 0.9), ("tile_size", 6)])
def test_backward_rejects_invalid_descriptor(field, value):
    desc, tun = _good()
    setattr(desc, field, value)
    assert _call_bwd(desc, tun) == binding.HMFSR_E_INVALID


def test_backward_rejects_invalid_tuning_and_pointers():
    desc, tun = _good()
    tun.k_shrink = 0.0
    assert _call_bwd(desc, tun) == binding.HMFSR_E_INVALID
    desc, tun = _good()
    assert _call_bwd(desc, tun, grad=None) == binding.HMFSR_E_INVALID
    assert _call_bwd(desc, tun, ptr=None) == binding.HMFSR_E_INVALID
    assert _call_bwd(desc, tun, grad=6) == binding.HMFSR_E_INVALID   # misaligned
    with pytest.raises(binding.HmfsrError):
        binding.hmfsr_merge_backward(desc, tun, 4, 4, 0, 4, 0, 4)


def test_stream_calls_validate_on_the_host():
    desc, tun = _good()
    L = binding.lib()
    bad = binding.make_desc(synth.Desc(4, 63, 96))   # odd height
    assert L.hmfsr_stream_begin(ctypes.byref(bad), ctypes.byref(tun), 4, 4, None) == binding.HMFSR_E_INVALID
    assert L.hmfsr_stream_begin(ctypes.byref(desc), ctypes.byref(tun), None, 4, None) == binding.HMFSR_E_INVALID
    assert L.hmfsr_stream_add(ctypes.byref(desc), ctypes.byref(tun), 4, 4, None, 4, None) == binding.HMFSR_E_INVALID
    assert L.hmfsr_stream_add(ctypes.byref(desc), ctypes.byref(tun), 4, 6, 4, 4, None) == binding.HMFSR_E_INVALID
    assert L.hmfsr_stream_end(ctypes.byref(desc), ctypes.byref(tun), 4, None, None) == binding.HMFSR_E_INVALID
    tun.k_shrink = 0.0
    assert L.hmfsr_stream_end(ctypes.byref(desc), ctypes.byref(tun), 4, 4, None) == binding.HMFSR_E_INVALID


def test_merge_rejects_misaligned_saved_buffer():
    desc, tun = _good()
    assert binding.lib().hmfsr_merge(ctypes.byref(desc), ctypes.byref(tun), 4, 4, 4, 12, None) == \
        binding.HMFSR_E_INVALID


def _align_call(desc, params, frames=8, motion=8, bm=None):
    return binding.lib().hmfsr_align(ctypes.byref(desc), ctypes.byref(params) if params is not None else None,
                                     frames, motion, bm, None)


@pytest.mark.parametrize("field,value", [
    ("levels", 0), ("levels", 7), ("radius_coarse", 0), ("radius_coarse", 9), ("radius_fine", 0),
    ("radius_fine", 9), ("lk_iterations", -1), ("lk_iterations", 17),
    ("gate", -1.0), ("gate", 1001.0), ("gate", float("nan")), ("gate", float("inf")),
])
def test_align_rejects_invalid_params(field, value):
    desc, _ = _good()
    params = binding.make_align_params()
    setattr(params, field, value)
    assert _align_call(desc, params) == binding.HMFSR_E_INVALID


def test_align_validates_descriptor_and_pointers():
    desc, _ = _good()
    p = binding.make_align_params()
    for field, value in (("tile_size", 66), ("tile_size", 128), ("n_frames", 0), ("height", 63)):
        d, _ = _good()
        setattr(d, field, value)
        assert _align_call(d, p) == binding.HMFSR_E_INVALID
    assert _align_call(desc, p, frames=None) == binding.HMFSR_E_INVALID
    assert _align_call(desc, p, motion=None) == binding.HMFSR_E_INVALID
    assert _align_call(desc, p, frames=2) == binding.HMFSR_E_INVALID      # not 4-byte aligned
    assert _align_call(desc, p, motion=4) == binding.HMFSR_E_INVALID      # not 8-byte aligned
    assert _align_call(desc, p, bm=4) == binding.HMFSR_E_INVALID
    with pytest.raises(binding.HmfsrError):
        bad = binding.make_align_params({"levels": 0})
        binding.hmfsr_align(desc, bad, 8, 8)
    assert binding.make_align_params({"lk_iterations": 5}).lk_iterations == 5


def test_noise_table_fields_validated():
    desc, tun = _good()
    desc.noise_bins = 4                      # bins without a table
    assert _call(desc, tun) == binding.HMFSR_E_INVALID
    desc, tun = _good()
    desc.noise_table = 8
    desc.noise_bins = 1                      # too few bins
    assert _call(desc, tun) == binding.HMFSR_E_INVALID
    desc.noise_bins = 70000
    assert _call(desc, tun) == binding.HMFSR_E_INVALID
    desc.noise_bins = 16
    desc.noise_table = 6                     # not 4-byte aligned
    assert _call(desc, tun) == binding.HMFSR_E_INVALID


def test_noise_table_and_auto_tuning_validate_on_the_host():
    L = binding.lib()
    desc, _ = _good()
    for bins, patches, table in ((1, 16, 8), (65537, 16, 8), (8, 0, 8), (8, 1 << 25, 8), (8, 16, None), (8, 16, 2)):
        assert L.hmfsr_noise_table(ctypes.byref(desc), bins, patches, 0, table, None) == binding.HMFSR_E_INVALID
    t = binding.hmfsr_tuning()
    assert L.hmfsr_auto_tuning(ctypes.byref(desc), None, ctypes.byref(t), None, None, None) == binding.HMFSR_E_INVALID
    assert L.hmfsr_auto_tuning(ctypes.byref(desc), 8, None, None, None, None) == binding.HMFSR_E_INVALID
    bad, _ = _good()
    bad.height = 63
    assert L.hmfsr_auto_tuning(ctypes.byref(bad), 8, ctypes.byref(t), None, None, None) == binding.HMFSR_E_INVALID


def test_desc_struct_has_no_padding():
    # the batch graph compares descriptors with memcmp
    assert ctypes.sizeof(binding.hmfsr_desc) == 14 * 4 + 8


def test_noalloc_refuses_bursts_beyond_its_scratch_on_the_host():
    """hmfsr_merge_noalloc checks the burst's map size against its static
    scratch before any HIP call (the dummy pointers are never used)."""
    d = synth.Desc(8, 3024, 4032, tile_size=16, scale=1.0)   # 12 MP x 8: ~390 MB of maps
    desc, tun = binding.make_desc(d), binding.make_tuning(synth.TUNING_SNR22)
    st = binding.lib().hmfsr_merge_noalloc(ctypes.byref(desc), ctypes.byref(tun), 16, 16, 16, None, None)
    assert st == binding.HMFSR_E_TOO_LARGE
    assert "static scratch" in binding.strerror(st)
    bad = binding.make_desc(synth.Desc(4, 64, 96, tile_size=16, scale=1.5))
    bad.height = 63
    assert binding.lib().hmfsr_merge_noalloc(ctypes.byref(bad), ctypes.byref(tun), 16, 16, 16, None,
                                             None) == binding.HMFSR_E_INVALID
