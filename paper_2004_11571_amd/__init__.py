"""MI355X-native partial modular polynomial evaluation (matrix method).

The compute path lives in the HIP/C++ shared library built from ``csrc/``;
``peval`` is its ctypes binding (argument marshalling only).
"""
