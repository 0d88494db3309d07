"""ctypes declarations of include/mlbm_probe.h: the streaming-read bandwidth
probe (libmlbm_probe.so), a measurement helper beside the method's library."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB_PATH = os.path.join(HERE, "libmlbm_probe.so")

PROBE_OK, PROBE_ERR_ARG, PROBE_ERR_HIP = 0, -1, -4
EXPORTS = ["mlbm_read_probe", "mlbm_probe_last_error"]


def load():
    try:
        import torch  # noqa: F401  (one HIP runtime per process: PyTorch's)
    except ImportError:
        pass
    if not os.path.exists(PROBE_LIB_PATH):
        raise ImportError(f"{PROBE_LIB_PATH} is missing: build it with python paper_2312_14789_amd/build.py")
    lib = ctypes.CDLL(PROBE_LIB_PATH)
    lib.mlbm_read_probe.restype = ctypes.c_int
    lib.mlbm_read_probe.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.mlbm_probe_last_error.restype = ctypes.c_char_p
    lib.mlbm_probe_last_error.argtypes = []
    return lib


def read_probe(lib, buf_ptr, nbytes, per_thread, out_ptr, stream_ptr):
    """mlbm_read_probe; raises RuntimeError on failure."""
    rc = lib.mlbm_read_probe(buf_ptr, nbytes, per_thread, out_ptr, stream_ptr)
    if rc != PROBE_OK:
        raise RuntimeError(f"mlbm_read_probe error {rc}: {lib.mlbm_probe_last_error().decode()}")
