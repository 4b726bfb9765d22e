"""MI355X (gfx950) electrostatic PIC-MCC step: HIP kernels behind a C ABI
(include/pic.h) and a thin ctypes binding (paper_2606_05893_amd.pic)."""
