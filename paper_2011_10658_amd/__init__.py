"""MI355X-native TTN node update for (3+1)D lattice QED.

The compute path lives in the HIP/C++ shared library `libqedttn.so`
(built in-tree by `build.py`); `lib` is its thin ctypes binding.  Importing
this package does not load the library; the first call into `lib` does,
and raises if the library is missing.
"""
