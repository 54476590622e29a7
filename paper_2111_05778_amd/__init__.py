"""Grid hopping polygonizer for MI355X: HIP kernels behind a C ABI (include/gh.h).

`native` is the ctypes binding of libgh.so (one Python function per C entry
point); `polygonize` allocates device buffers with torch and sequences the
calls.  Importing either fails when libgh.so has not been built.
"""
__all__ = ["native", "polygonize"]
