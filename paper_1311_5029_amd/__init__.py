"""MI355X-native Oktay-Kronfeld operator and BiCGStab inverter.

The compute path is the HIP library ``libokinv.so`` behind the C-ABI declared
in ``include/okinv.h``; ``paper_1311_5029_amd.okinv`` is its thin ctypes
binding.  Importing this package loads nothing: import ``okinv`` explicitly.
"""
