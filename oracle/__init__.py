"""Plain FP64 CPU oracle of the FC-Gram pseudospectral step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything in this directory; only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path: the only common module is ``workloads`` (seeded synthetic
inputs, which holds none of the method's arithmetic).

Modules
-------
fft       The discrete Fourier transforms, written out: the definition as a
          matrix product, and the same sums by Cooley-Tukey splitting.
fc_table  Gram basis and blend-to-zero continuation tables (App. B).
fcgram    FC-Gram continuation of lines and FC spectral derivatives (Sec. 3).
ns        The time-splitting Runge-Kutta step with the pressure projection
          (Sec. 4.1-4.4), the Boussinesq extension (Sec. 7) and the channel
          forcing (Sec. 6).

Everything is plain numpy in float64.  No FFT library is used: the
transforms are the oracle's own (``fft``), pinned against the DFT evaluated
term by term; numpy's matrix product is the only library primitive.
"""
