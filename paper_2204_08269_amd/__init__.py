"""MI355X-native joint time-frequency scattering (arxiv 2204.08269) and its gradient."""
from ._lib import JTFSError, load  # noqa: F401


def JTFS(*args, **kwargs):
    from .jtfs import JTFS as _J
    return _J(*args, **kwargs)
