"""dlmi: MI355X (gfx950) patch featurisation and exact similarity joins.

The data-parallel hot path of the DeepLens query layer (Krishnan et al.,
CIDR 2019): colour-histogram featurisation of image patches and eps-range /
top-k joins under L2 distance, behind the C ABI of libdlmi.so
(include/dlmi.h).  This package is the thin Python binding: `ops` marshals
torch device tensors into the C calls; `synth` draws seeded synthetic
inputs; `build` compiles the library.  Submodules are imported on demand.
"""
__all__ = ["ops", "synth", "build"]
