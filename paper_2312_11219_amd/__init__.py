"""gaca: 3-way (generalised) ACA of Laplace-domain BEM tensors on MI355X (gfx950).

Thin Python binding over the C ABI in ``include/gaca.h`` (``libgaca.so``): argument
marshalling only; every step of the build and the apply runs in the HIP library.
PyTorch is used for device memory and streams.
"""
from ._binding import (Context, HMatrix, Problem, compress_tensor, gcq_contour, lib_path,
                       load_library, options_default, partition_host)

__all__ = ["Context", "Problem", "HMatrix", "compress_tensor", "partition_host",
           "options_default", "load_library", "lib_path", "gcq_contour"]
