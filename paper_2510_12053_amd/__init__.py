"""Coordinate Condensation on AMD MI355X: a C-ABI library (libccgpu.so, HIP
kernels for gfx950) and its Python binding ``ccgpu``."""
