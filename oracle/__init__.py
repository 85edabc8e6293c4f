"""FP64 CPU oracle for JTFS -- test infrastructure only (see jtfs_oracle)."""
from .jtfs_oracle import *  # noqa: F401,F403
from .jtfs_oracle import Plan, jtfs, jtfs_vjp, jtfs_direct, fft, ifft, dft_direct  # noqa: F401
