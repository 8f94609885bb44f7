"""Torch-tensor front end of libhmfsr: shape/dtype checks and marshalling.

PyTorch supplies device memory and the current stream; the merge itself runs
in the library's HIP kernels. Tensors must live on a ROCm device.
"""
from __future__ import annotations

import torch

from . import binding


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_inputs(frames: torch.Tensor, motion: torch.Tensor, desc):
    if not frames.is_cuda or not motion.is_cuda:
        raise ValueError("frames and motion must be device tensors (no CPU path exists)")
    if frames.dtype not in (torch.uint16, torch.int16):
        raise ValueError(f"frames must be uint16 (or an int16 view), got {frames.dtype}")
    if motion.dtype != torch.float32:
        raise ValueError(f"motion must be float32, got {motion.dtype}")
    n, h, w = desc.n_frames, desc.height, desc.width
    ty, tx = -(-h // desc.tile_size), -(-w // desc.tile_size)
    if tuple(frames.shape) != (n, h, w):
        raise ValueError(f"frames shape {tuple(frames.shape)} != {(n, h, w)}")
    if tuple(motion.shape) != (n, ty, tx, 2):
        raise ValueError(f"motion shape {tuple(motion.shape)} != {(n, ty, tx, 2)}")
    if not frames.is_contiguous() or not motion.is_contiguous():
        raise ValueError("frames and motion must be contiguous")
    if frames.device != motion.device:
        raise ValueError("frames and motion must be on one device")


def _check_out(t: torch.Tensor | None, shape, device, what):
    if t is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    if tuple(t.shape) != tuple(shape) or t.dtype != torch.float32 or not t.is_contiguous() \
            or t.device != device:
        raise ValueError(f"{what} must be a contiguous float32 tensor of shape {tuple(shape)} on {device}")
    return t


def merge(frames: torch.Tensor, motion: torch.Tensor, desc, tuning,
          out: torch.Tensor | None = None, saved: torch.Tensor | None = None) -> torch.Tensor:
    """Merge one burst; returns float32 [3][OH][OW] on the frames' device.
    ``saved`` (float32 [12][OH][OW], see ``saved_buffer``), if given, receives
    the normaliser the adjoint can reuse."""
    _check_inputs(frames, motion, desc)
    out = _check_out(out, (3, desc.out_height, desc.out_width), frames.device, "out")
    if saved is not None:
        _check_out(saved, (12, desc.out_height, desc.out_width), frames.device, "saved")
    with torch.cuda.device(frames.device):
        binding.hmfsr_merge(binding.make_desc(desc), binding.make_tuning(tuning),
                            frames.data_ptr(), motion.data_ptr(), out.data_ptr(),
                            0 if saved is None else saved.data_ptr(), _stream(frames.device))
    return out


def align(frames: torch.Tensor, desc, params=None, motion: torch.Tensor | None = None,
          block_match: bool = False):
    """Per-tile alignment vectors of every frame against the base frame
    (float32 [N][TY][TX][2], the layout ``merge`` reads). ``params``: dict of
    hmfsr_align_params fields (missing ones take the defaults). With
    ``block_match`` also returns the integer block-matching vectors
    (int32 [N][TY][TX][2], half-resolution pixels)."""
    if not frames.is_cuda:
        raise ValueError("frames must be a device tensor (no CPU path exists)")
    if frames.dtype not in (torch.uint16, torch.int16):
        raise ValueError(f"frames must be uint16 (or an int16 view), got {frames.dtype}")
    n, h, w = desc.n_frames, desc.height, desc.width
    if tuple(frames.shape) != (n, h, w) or not frames.is_contiguous():
        raise ValueError(f"frames must be contiguous of shape {(n, h, w)}")
    shape = (n, -(-h // desc.tile_size), -(-w // desc.tile_size), 2)
    motion = _check_out(motion, shape, frames.device, "motion")
    bm = torch.empty(shape, dtype=torch.int32, device=frames.device) if block_match else None
    with torch.cuda.device(frames.device):
        binding.hmfsr_align(binding.make_desc(desc), binding.make_align_params(params),
                            frames.data_ptr(), motion.data_ptr(), 0 if bm is None else bm.data_ptr(),
                            _stream(frames.device))
    return (motion, bm) if block_match else motion


def noise_table(desc, device, bins: int = 64, patches: int = 4096, seed: int = 0) -> torch.Tensor:
    """Monte-Carlo noise table float32 [bins][4] for the descriptor's noise
    model and raw range (Sec. 5.2.2); set it as ``desc.noise_table``."""
    table = torch.empty((bins, 4), dtype=torch.float32, device=device)
    with torch.cuda.device(table.device):
        plain = dataclass_replace_table(desc, None)
        binding.hmfsr_noise_table(binding.make_desc(plain), bins, patches, seed, table.data_ptr(),
                                  _stream(table.device))
    return table


def dataclass_replace_table(desc, table):
    """A copy of ``desc`` with another noise table (descriptors with a
    ``replace`` method, else the same object when no table is involved)."""
    if hasattr(desc, "replace"):
        return desc.replace(noise_table=table)
    if getattr(desc, "noise_table", None) is not None:
        raise ValueError("descriptor has a noise table but no replace()")
    return desc


def auto_tuning(frames: torch.Tensor, desc):
    """SNR-dependent tuning of the burst (Sec. 7.2, S.2): returns
    (synth.Tuning, suggested tile size, SNR)."""
    from .synth import Tuning
    if not frames.is_cuda:
        raise ValueError("frames must be a device tensor (no CPU path exists)")
    with torch.cuda.device(frames.device):
        tun, tile, snr = binding.hmfsr_auto_tuning(binding.make_desc(desc), frames.data_ptr(),
                                                   _stream(frames.device))
    vals = {f: getattr(tun, f) for f, _ in binding.hmfsr_tuning._fields_}
    return Tuning(**vals), tile, snr


def merge_raw(frames: torch.Tensor, desc, tuning, params=None) -> torch.Tensor:
    """Raw burst to RGB: ``align`` then ``merge``."""
    return merge(frames, align(frames, desc, params), desc, tuning)


def saved_buffer(desc, device) -> torch.Tensor:
    """A buffer for the forward's normaliser: 12 words per output pixel (three
    float64 planes of C, three float32 planes each of the denominator and the
    reference exponent)."""
    return torch.empty((12, desc.out_height, desc.out_width), dtype=torch.float32, device=device)


def merge_backward(frames: torch.Tensor, motion: torch.Tensor, desc, tuning,
                   grad_out: torch.Tensor, saved: torch.Tensor | None = None):
    """Adjoint of ``merge`` for dL/dC = grad_out: returns (grad_tuning float32
    [9] in ``binding.GRAD_NAMES`` order, grad_motion float32 [N][TY][TX][2]),
    both on the frames' device."""
    _check_inputs(frames, motion, desc)
    dev = frames.device
    shape = (3, desc.out_height, desc.out_width)
    grad_out = grad_out.to(device=dev, dtype=torch.float32).contiguous()
    if tuple(grad_out.shape) != shape:
        raise ValueError(f"grad_out shape {tuple(grad_out.shape)} != {shape}")
    if saved is not None:
        _check_out(saved, (12,) + shape[1:], dev, "saved")
    g_tun = torch.empty(9, dtype=torch.float32, device=dev)
    g_mot = torch.empty_like(motion)
    with torch.cuda.device(dev):
        binding.hmfsr_merge_backward(binding.make_desc(desc), binding.make_tuning(tuning),
                                     frames.data_ptr(), motion.data_ptr(),
                                     0 if saved is None else saved.data_ptr(), grad_out.data_ptr(),
                                     g_tun.data_ptr(), g_mot.data_ptr(), _stream(dev))
    return g_tun, g_mot


class StreamingMerge:
    """Frames added one at a time into a fixed-size accumulator state
    ([9][OH][OW] float32), then normalised: memory does not grow with the
    frame count. Adding the frames in the order ``merge`` visits them (base
    frame first, then the others by index) reproduces ``merge`` with the
    64 x 16 tile shape bit for bit."""

    def __init__(self, base_frame: torch.Tensor, desc, tuning):
        if not base_frame.is_cuda or base_frame.dtype not in (torch.uint16, torch.int16) \
                or tuple(base_frame.shape) != (desc.height, desc.width) or not base_frame.is_contiguous():
            raise ValueError("base_frame must be a contiguous uint16 device tensor [H][W]")
        self.desc, self.tuning, self.base = desc, tuning, base_frame
        self.dev = base_frame.device
        self.state = torch.empty((9, desc.out_height, desc.out_width), dtype=torch.float32, device=self.dev)
        self.frames = 1
        with torch.cuda.device(self.dev):
            binding.hmfsr_stream_begin(binding.make_desc(desc), binding.make_tuning(tuning),
                                       base_frame.data_ptr(), self.state.data_ptr(), _stream(self.dev))

    def add(self, frame: torch.Tensor, motion: torch.Tensor) -> None:
        d = self.desc
        if frame.device != self.dev or frame.dtype != self.base.dtype or tuple(frame.shape) != (d.height, d.width) \
                or not frame.is_contiguous():
            raise ValueError("frame must be a contiguous tensor like the base frame")
        ty, tx = -(-d.height // d.tile_size), -(-d.width // d.tile_size)
        if motion.device != self.dev or motion.dtype != torch.float32 or tuple(motion.shape) != (ty, tx, 2) \
                or not motion.is_contiguous():
            raise ValueError(f"motion must be a contiguous float32 device tensor {(ty, tx, 2)}")
        with torch.cuda.device(self.dev):
            binding.hmfsr_stream_add(binding.make_desc(d), binding.make_tuning(self.tuning),
                                     self.base.data_ptr(), frame.data_ptr(), motion.data_ptr(),
                                     self.state.data_ptr(), _stream(self.dev))
        self.frames += 1

    def result(self, out: torch.Tensor | None = None) -> torch.Tensor:
        d = self.desc
        out = _check_out(out, (3, d.out_height, d.out_width), self.dev, "out")
        with torch.cuda.device(self.dev):
            binding.hmfsr_stream_end(binding.make_desc(d), binding.make_tuning(self.tuning),
                                     self.state.data_ptr(), out.data_ptr(), _stream(self.dev))
        return out


TUNING_FIELDS = binding.GRAD_NAMES + ("m_th",)


class _TuningView:
    """Attribute view of a 10- or 11-vector of tuning values (hmfsr_tuning
    order; the 11th, hf_ratio, defaults to 0)."""

    def __init__(self, values):
        self.hf_ratio = 0.0
        for name, v in zip(TUNING_FIELDS + ("hf_ratio",), values):
            setattr(self, name, float(v))


class HmfsrMerge(torch.autograd.Function):
    """C = merge(frames, motion, tuning) with gradients for motion and the
    tuning vector [k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink, s, t,
    s_motion, m_th(, hf_ratio)] (the thresholds m_th and hf_ratio get zero).
    The forward keeps the normaliser of
    eq. (1) so that the backward needs no second forward."""

    @staticmethod
    def forward(ctx, frames, motion, tuning_vec, desc):
        tun = _TuningView(tuning_vec.detach().to("cpu", torch.float32).tolist())
        motion_c = motion.detach().contiguous()
        saved = saved_buffer(desc, frames.device)
        out = merge(frames, motion_c, desc, tun, saved=saved)
        ctx.save_for_backward(frames, motion_c, saved)
        ctx.desc, ctx.tun = desc, tun
        ctx.tuning_meta = (tuning_vec.device, tuning_vec.dtype)
        ctx.n_tuning = tuning_vec.numel()
        return out

    @staticmethod
    def backward(ctx, grad_out):
        frames, motion, saved = ctx.saved_tensors
        g_tun, g_mot = merge_backward(frames, motion, ctx.desc, ctx.tun, grad_out, saved=saved)
        dev, dt = ctx.tuning_meta
        extra = ctx.n_tuning - g_tun.numel()     # m_th (and hf_ratio): thresholds, no gradient
        g_vec = torch.cat([g_tun, g_tun.new_zeros(extra)]).to(device=dev, dtype=dt)
        return None, g_mot, g_vec, None


def merge_autograd(frames, motion, tuning_vec, desc):
    """Differentiable merge (see ``HmfsrMerge``)."""
    return HmfsrMerge.apply(frames, motion, tuning_vec, desc)


def merge_maps(frames: torch.Tensor, motion: torch.Tensor, desc, tuning) -> dict:
    """Per-frame intermediate maps: omega [N][3][h][w] f64, robust and
    robust_min [N][h][w] f32, s_tile [N][TY][TX] f32."""
    _check_inputs(frames, motion, desc)
    dev = frames.device
    n, h, w = desc.n_frames, desc.height // 2, desc.width // 2
    ty, tx = -(-desc.height // desc.tile_size), -(-desc.width // desc.tile_size)
    res = dict(omega=torch.empty((n, 3, h, w), dtype=torch.float64, device=dev),
               robust=torch.empty((n, h, w), dtype=torch.float32, device=dev),
               robust_min=torch.empty((n, h, w), dtype=torch.float32, device=dev),
               s_tile=torch.empty((n, ty, tx), dtype=torch.float32, device=dev))
    with torch.cuda.device(dev):
        binding.hmfsr_merge_maps(binding.make_desc(desc), binding.make_tuning(tuning),
                                 frames.data_ptr(), motion.data_ptr(), res["omega"].data_ptr(),
                                 res["robust"].data_ptr(), res["robust_min"].data_ptr(),
                                 res["s_tile"].data_ptr(), _stream(dev))
    return res


def merge_batch(bursts, outs=None) -> list:
    """Merge a list of (frames, motion, desc, tuning) tuples in one graph launch.
    Returns the output tensors (allocated unless given)."""
    if outs is None:
        outs = [torch.empty((3, d.out_height, d.out_width), dtype=torch.float32, device=f.device)
                for f, m, d, t in bursts]
    dev = bursts[0][0].device
    for (f, m, d, t), o in zip(bursts, outs):
        _check_inputs(f, m, d)
        if f.device != dev or o.device != dev or tuple(o.shape) != (3, d.out_height, d.out_width) \
                or o.dtype != torch.float32 or not o.is_contiguous():
            raise ValueError("every burst and output must be on one device, outputs [3][OH][OW] float32")
    with torch.cuda.device(dev):
        binding.hmfsr_merge_batch([binding.make_desc(d) for f, m, d, t in bursts],
                                  [binding.make_tuning(t) for f, m, d, t in bursts],
                                  [f.data_ptr() for f, m, d, t in bursts],
                                  [m.data_ptr() for f, m, d, t in bursts],
                                  [o.data_ptr() for o in outs], _stream(dev))
    return outs


def batch_plan(device) -> dict:
    """Items and workgroups of the persistent launches of the last batch graph
    captured on ``device``."""
    with torch.cuda.device(device):
        return binding.hmfsr_batch_plan()


def autotune(frames: torch.Tensor, motion: torch.Tensor, desc, tuning,
             out: torch.Tensor | None = None):
    """Run the tile-shape autotuner on one burst; returns (chosen index, output)."""
    _check_inputs(frames, motion, desc)
    if out is None:
        out = torch.empty((3, desc.out_height, desc.out_width), dtype=torch.float32,
                          device=frames.device)
    with torch.cuda.device(frames.device):
        v = binding.hmfsr_autotune(binding.make_desc(desc), binding.make_tuning(tuning),
                                   frames.data_ptr(), motion.data_ptr(), out.data_ptr(),
                                   _stream(frames.device))
    return v, out
