"""MI355X-native coupled-cluster doubles (CCD) for pure neutron matter.

The compute path is libccd.so (HIP kernels for gfx950, C ABI in include/ccd.h);
this package only binds it.  Importing the package fails if the library has not
been built (python -m paper_1611_06765_amd.build_lib).
"""
from . import ccd  # noqa: F401
from .ccd import Context, problem, canonical_index  # noqa: F401
