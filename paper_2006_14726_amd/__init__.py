"""MI355X-native splat ray tracer: the client-side path of image-warping
remote volume rendering with ray tracing (arXiv 2006.14726).

2.5D RGBA + depth pixels are unprojected into spheres (Eq. 1), a linear BVH
is built over them, and a new view is ray traced through them with exact
front-to-back compositing.  Every step runs in the HIP kernels of
``libsplat.so`` (gfx950); torch provides device memory and streams.
"""
from . import _lib
from ._lib import (SPLAT_ALPHA_CONSTANT, SPLAT_ALPHA_SOFT, SPLAT_F16, SPLAT_F32, SPLAT_RADIUS_FOOTPRINT,
                   SPLAT_RADIUS_INTERVAL, SPLAT_RADIUS_OPACITY, SPLAT_RADIUS_SPHEROID, SPLAT_STATUS_CORRUPT,
                   SPLAT_STATUS_STACK, SplatError)
from .render import (BVH, Spheres, TraceOptions, accumulate, alloc_bvh, alloc_grads, alloc_spheres, build_bvh,
                     build_bvh_from_samples,
                     decode_samples, zero_grads,
                     encode_samples, raymarch, render, spheres_from_tensors, trace, trace_backward, trace_noalloc, unproject,
                     unproject_policy)

__all__ = ["BVH", "Spheres", "TraceOptions", "SplatError", "alloc_bvh", "alloc_spheres", "build_bvh",
           "build_bvh_from_samples", "raymarch", "render",
           "spheres_from_tensors", "trace", "trace_backward", "trace_noalloc", "unproject", "encode_samples", "decode_samples", "accumulate", "unproject_policy", "alloc_grads", "zero_grads", "SPLAT_ALPHA_CONSTANT",
           "SPLAT_RADIUS_FOOTPRINT", "SPLAT_RADIUS_OPACITY", "SPLAT_RADIUS_INTERVAL", "SPLAT_RADIUS_SPHEROID",
           "SPLAT_ALPHA_SOFT", "SPLAT_F16", "SPLAT_F32", "SPLAT_STATUS_CORRUPT", "SPLAT_STATUS_STACK", "load_library"]


def load_library():
    """Load libsplat.so (raises ImportError if it was not built)."""
    return _lib.load()
