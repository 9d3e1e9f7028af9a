"""MI355X (gfx950) fractal image encoder: the range-to-domain block search of
Salarian & Miar Naimi's modified fast fractal coder, as HIP kernels behind a
C ABI (include/fic.h).  ``fic`` is the Python binding; ``synth`` and
``configs`` provide seeded inputs and the workload presets."""
__all__ = ["fic", "synth", "configs"]
