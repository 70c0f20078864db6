"""The warm-start network library loads without a GPU, exports every symbol
its header declares, and validates arguments on the host."""
import ctypes
import os
import re

from paper_2312_10615_amd import unet as U

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokes_unet.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t)\s+(unet_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = U.load_library()
    names = declared_functions()
    assert "unet_conv3" in names and "unet_conv3_wgrad" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(U.EXPORTS) == names


def test_packed_sizes():
    # cin=16 -> one 16-channel chunk: 27*2 = 54 K octets -> 14 k-steps of 4 octets;
    # cout=32 -> two 16-wide output tiles; 64 lanes x 8 values each
    assert U.unet_packed_elems(16, 32, False) == 14 * 2 * 64 * 8
    # transposed (input gradient): 32 input channels (one 32-channel chunk = 27 k-steps), 16 outputs
    assert U.unet_packed_elems(16, 32, True) == 27 * 1 * 64 * 8
    # 96 input channels: three 32-channel chunks
    assert U.unet_packed_elems(96, 32, False) == 3 * 27 * 2 * 64 * 8
    # unsupported shapes report 0
    assert U.unet_packed_elems(12, 16, False) == 0
    assert U.unet_packed_elems(16, 24, False) == 0


def test_invalid_arguments_are_rejected_without_a_device():
    lib = U.load_library()
    src = U.Source(U.SRC_DIRECT, 4, 4, 4, 16, 0, 0, 0)  # null input pointer
    assert lib.unet_conv3(ctypes.byref(src), 16, None, None, 1, 0, None, None) == U.UNET_EINVAL
    src.src0 = 16
    src.channels = 12  # not a multiple of 8
    assert lib.unet_conv3(ctypes.byref(src), 16, ctypes.c_void_p(16), None, 1, 0, ctypes.c_void_p(16),
                          None) == U.UNET_EINVAL
    cat = U.Source(U.SRC_CAT_UP, 5, 4, 4, 48, 32, 16, 32)  # odd grid cannot take an upsampled input
    assert lib.unet_conv3(ctypes.byref(cat), 16, ctypes.c_void_p(16), None, 1, 0, ctypes.c_void_p(16),
                          None) == U.UNET_EINVAL
    assert lib.unet_adam(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) == U.UNET_EINVAL


def test_workspace_queries():
    x = U.Source(U.SRC_DIRECT, 16, 16, 16, 16, 0, 16, 0)
    assert U.unet_wgrad_workspace_bytes(x, 16) >= 4 * 27 * 16 * 16
    assert U.unet_head_workspace_bytes(16 ** 3) >= 4 * 68
    assert U.unet_mse_workspace_bytes(16 ** 3) > 0
