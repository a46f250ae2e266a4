"""MI355X-native stereo reprojection: one rendered eye (RGBA8 + FP32 depth) to
the other eye, after "You Only Render Once" (Sections 5-7).

The compute path is the C-ABI library ``libyoro.so`` (HIP kernels for gfx950,
declared in ``include/yoro.h``); ``paper_2506_15183_amd.yoro`` is its thin
Python binding (torch tensors in, device pointers and the current stream
out).  ``paper_2506_15183_amd.scenes`` makes the seeded synthetic inputs.

Nothing is imported eagerly, so the scene generator works on machines with
no GPU and no built HIP library.
"""

__all__ = ["yoro", "scenes"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
