"""On-demand decoding of baseline-JPEG textures during deferred shading, for
AMD Instinct MI355X (gfx950): a C-ABI library (libjpt.so, include/jpt.h) of
hand-written HIP kernels, with a thin Python binding (jpt) and seeded
synthetic inputs (synth)."""
