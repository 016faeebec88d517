"""MI355X (gfx950) dual heterogeneous island GA for the flexible flow shop.

The hot path (decode, cellular and pseudo generation step, migration) runs in
hand-written HIP kernels behind the C ABI of include/ffs.h; `binding` is the
ctypes layer with the same entry points, PyTorch only supplies device memory
and the stream.
"""
from .binding import Context, FFSError, library_path, load_library  # noqa: F401
