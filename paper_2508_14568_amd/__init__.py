"""MI355X-native Leuvenshtein encrypted edit distance (arXiv 2508.14568).

``lvs`` is the Python binding of ``liblvs.so`` (C ABI in ``include/lvs.h``):
host key generation and encryption, and on the GPU the programmable
bootstraps of the single-lookup cell update, the 2-PBS ASCII equality, the
anti-diagonal wavefront driver and the one-cleartext-string preprocessing.
"""
from . import lvs  # noqa: F401

__all__ = ["lvs"]
