"""MI355X-native coupled-cluster doubles (CCD) for pure neutron matter.

The compute path is libccd.so (HIP kernels for gfx950, C ABI in include/ccd.h);
this package only binds it.  The binding is loaded on first use, so that the
build step (python -m paper_1611_06765_amd.build_lib) runs before a library
exists; using the binding fails loudly if the library has not been built.
"""
import importlib

_LAZY = {"Context": "ccd", "problem": "ccd", "canonical_index": "ccd"}


def __getattr__(name):
    if name in ("ccd", "warmstart"):
        return importlib.import_module(f".{name}", __name__)
    if name in _LAZY:
        return getattr(importlib.import_module(f".{_LAZY[name]}", __name__), name)
    raise AttributeError(name)
