"""ssmap: LADMM spatial-spectral partial-volume mapping on AMD MI355X (gfx950).

The solver lives in libssmap.so (C ABI in include/ssmap.h); `_ffi` is its
ctypes binding and `synth` draws seeded synthetic problems. Importing the
package loads nothing; `load()` opens the library and fails loudly when it
has not been built.
"""
__all__ = ["load"]


def load():
    from . import _ffi
    return _ffi.load()
