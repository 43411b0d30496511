"""MI355X (gfx950) damped-acoustic finite-difference propagator.

The hot path — the leapfrog stencil with fused source injection and receiver
sampling, its adjoint, the imaging-condition gradient and checkpointing —
lives in the HIP library ``_build/libwave.so`` behind the C ABI of
``include/wave.h``.  ``api`` holds the PyTorch-facing wrappers and the
autograd function; ``synth`` makes seeded synthetic inputs.
"""
__version__ = "0.1.0"


def __getattr__(name):
    # the torch-facing API is loaded on first use, so that importing the
    # package (e.g. for ``synth``) does not require torch or the library
    if name in ("Geometry", "forward", "adjoint", "backward", "gradient", "WaveFn",
                "wave_apply", "checkpoint_bytes"):
        import importlib
        return getattr(importlib.import_module(__name__ + ".api"), name)
    raise AttributeError(name)
