"""MI355X phaseless-AFQMC walker-step library: HIP kernels behind a C ABI
(include/afq.h) and a thin ctypes binding (paper_2403_02542_amd.afq)."""
