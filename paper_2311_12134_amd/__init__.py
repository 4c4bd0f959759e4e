"""MI355X (gfx950) implementation of the LSMS tau-solve + Kubo-Greenwood hot path.

The compute lives in liblsms_kkr.so (HIP kernels + C ABI, see include/lsms_kkr.h);
this package only loads it and marshals arguments.
"""

from .api import Context, KuboSigma, Liz, build_liz, gaunt_table  # noqa: F401
