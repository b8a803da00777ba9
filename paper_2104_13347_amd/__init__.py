"""MI355X-native image-source-method room impulse responses (HIP, gfx950).

The product is ``libism.so`` (C-ABI, declared in ``include/ism.h``); the
``ism`` module is a thin ctypes binding that passes torch device pointers and
streams through.  ``scenes`` draws seeded synthetic inputs.  Nothing here is
imported eagerly: loading the library happens on first use and fails loudly
if it was not built.
"""
__all__ = ["ism", "scenes"]
