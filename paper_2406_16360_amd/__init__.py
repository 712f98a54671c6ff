"""MI355X-native differentiable path tracer with reservoir-resampled
environment lighting (the rendering hot path of MIRReS, arXiv 2406.16360).

The renderer itself lives in the HIP library under csrc/ behind a C ABI
(include/mirres.h); `paper_2406_16360_amd.mirres` is the thin Python binding.
Submodules are imported lazily so that `paper_2406_16360_amd.synth` (seeded
inputs only) can be used without loading the GPU library.
"""
__all__ = ["synth", "mirres"]
