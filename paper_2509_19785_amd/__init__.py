"""MI355X-native L-tsNET gradient: HIP kernels behind a C ABI (libtsnet.so).

``api`` holds torch-facing wrappers, ``_lib`` the one-to-one ctypes binding,
``autograd`` the cost as a torch.autograd.Function. Importing ``api`` or
``_lib`` raises ImportError if the library has not been built
(``python -m paper_2509_19785_amd.build``); there is no CPU fallback.
"""

__all__ = ["api", "autograd", "build"]
