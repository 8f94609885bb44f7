"""MI355X-native kernel-regression burst merge (handheld multi-frame super-resolution).

The hot path lives in ``libhmfsr.so`` (hand-written HIP for gfx950, C ABI in
``include/hmfsr.h``). ``binding`` marshals arguments to it; ``torch_ops`` wraps
it for torch tensors; ``synth`` draws seeded synthetic bursts. Nothing here is
imported eagerly so that importing the package never loads the GPU library.
"""
__all__ = ["binding", "torch_ops", "synth", "build"]
