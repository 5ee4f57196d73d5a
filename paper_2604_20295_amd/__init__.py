"""MI355X-native ETac tactile step: HIP kernels for gfx950 behind the C ABI
of include/etac.h (libetac.so), a ctypes binding with the same names
(`_native`: Plan, MeshSet and one function per C call), torch.autograd
bindings (`autograd.ETacStep` for primitives, `autograd.ETacMeshStep` for
scenes with triangle-mesh objects) and the Eq. 3 calibration loop
(`calibrate`)."""
from . import _native  # noqa: F401
