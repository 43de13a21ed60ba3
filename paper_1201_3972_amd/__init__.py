"""MI355X-native FNR impulse filter for infrared frames.

The filter (detect impulses as window extremes, replace them by the window
median) runs in hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/irfilter.h``.  ``paper_1201_3972_amd.irfilter`` is the thin ctypes
binding of that library; ``paper_1201_3972_amd.synth`` draws seeded inputs.
Importing this package loads nothing: the binding loads the shared library on
first use and raises if it is missing.
"""
