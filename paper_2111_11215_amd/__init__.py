"""MI355X (gfx950) implementation of the fine-stage per-ray training step of
direct voxel-grid radiance-field optimisation (Sun, Sun and Chen,
arXiv 2111.11215): ray-box clipping, uniform sampling with coarse alpha-mask
skipping, post-activated density and feature interpolation, a shallow
view-conditioned MLP on matrix cores, front-to-back compositing, the adjoint
that walks each ray from its end, and Adam; plus a learned segment proposal.

The compute lives in the HIP library ``libdvgo.so`` (C ABI in
``include/dvgo.h``); this package only marshals torch tensors into it.
"""

__all__ = ["api", "train"]
