"""MI355X-native BPFA blind inpainting (Gibbs sweep on hand-written HIP kernels).

``paper_2311_15061_amd.bpfa`` binds the C ABI of ``_lib/libbpfa.so``
(declared in ``include/bpfa.h``); importing it fails when the library has not
been built.  ``metrics`` holds the binary64 image-quality measures used to
report results.
"""
from . import metrics  # noqa: F401
