"""MI355X-native object-aware differentiable Gaussian rasterization (DQO-MAP hot path).

The compute path is the HIP library `libdqo.so` (built from `csrc/`), reached
through the thin ctypes binding in `binding.py`; `scenes.py` holds seeded
synthetic inputs.  Nothing is loaded at import time.
"""
__all__ = ["binding", "scenes"]
