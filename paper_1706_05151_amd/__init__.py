"""MI355X-native exact triangle counting (degree-ordered NodeIteratorN, arXiv 1706.05151).

The compute path is the HIP library ``libtc.so`` behind the C ABI of
``include/tc.h``; :mod:`paper_1706_05151_amd.tc` is its Python binding.
"""
from .tc import Graph, TCError, get_option, lib, set_option  # noqa: F401

__all__ = ["Graph", "TCError", "get_option", "set_option", "lib"]
