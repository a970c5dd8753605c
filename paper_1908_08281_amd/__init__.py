"""MI355X-native hypergraph ranking solves (HIP kernels behind a C ABI).

The compute lives in ``libhgl.so`` (``csrc/*.hip``, built for gfx950 by
``python -m paper_1908_08281_amd.build``); ``hgl`` is the torch-facing
binding.  Importing this package does not load the library; the first call
into ``hgl`` does, and raises if it is not built.
"""
__all__ = ["hgl"]
