"""MI355X (gfx950) APAX numerical encoder, decoder and profiler.

The compute runs in libapax.so (hand-written HIP); `apax` is its Python
binding.  Importing the binding raises if the library is not built.
"""
