"""CPU oracle for the inverse spherical harmonic transform (alm2map).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path (``paper_1010_1260_amd``) and never imports it.

Contents
--------
``sht_oracle.c``  plain FP64 C: Legendre functions, Delta_m(theta) and the
                  transposed Legendre stage (Sec. 2.1-2.2.2, Algorithms 1-2).
``ref``           Python wrapper and the per-ring Fourier steps (Eq. Delta2map
                  with the wrap-around rule of Sec. 2.2.2), using numpy.fft as
                  the FFT primitive, plus a literal direct-sum variant.
``brute``         exact-rational spherical harmonics for small l_max (brute
                  force summation at every pixel).
"""
