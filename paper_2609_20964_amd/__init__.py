"""MI355X-native grid-Poisson SDF reconstruction (the Warp-Geo hot path).

libwgeo.so (HIP, gfx950) holds every kernel; this package is its thin Python
face: ``Recon`` (one resident grid), ``reconstruct`` (autograd function with the
hand-written adjoint) and ``Server`` (continuous batching).
"""
from ._lib import LIB_PATH, WgError  # noqa: F401


def __getattr__(name):
    if name in ("Recon", "reconstruct"):
        from . import recon
        return getattr(recon, name)
    if name == "Server":
        from .serving import Server
        return Server
    raise AttributeError(name)
