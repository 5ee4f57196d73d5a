"""MI355X-native ETac tactile step: HIP kernels for gfx950 behind the C ABI
of include/etac.h (libetac.so), a ctypes binding with the same names
(`_native`) and a torch.autograd binding (`autograd.ETacStep`)."""
from . import _native  # noqa: F401
