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
    assert binding.hmfsr_version() == 110
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
