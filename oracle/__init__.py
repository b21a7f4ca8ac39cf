"""FP64 CPU oracle for the NeRF-SLAM mapping step (Rosinol, Leonard,
Carlone, "NeRF-SLAM: Real-Time Dense Monocular SLAM with Neural Radiance
Fields").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP library
or its Python binding.

It is a plain, slow, obviously-correct implementation written from the
paper: the mapping loss (Sec. 3.2, Eq. 3), the Sigma_D-weighted depth loss
(Eq. 4), rendered depth (Eq. 5), transmittance (Eq. 6), the photometric loss
(Eq. 7) and the composited colour (Sec. 3.2, after Eq. 7), on a hash-grid
field whose details the paper defers to Instant-NGP (Sec. 3.2, Sec. 3.4).
Arithmetic is IEEE double precision throughout, with one deliberate
exception: sample positions decide integer cell and corner indices, so they
are formed in single precision with a fixed operation order (``rays.py``),
which the GPU path reproduces; every continuous quantity after that is FP64.

Every gradient is returned with a *magnitude*: the same reverse-mode
expression evaluated with absolute values (subtractions become sums).  A
float32 implementation that sums the same terms in any order lands within a
small multiple of ``u * magnitude`` of the exact value, so parity tests bound
``|gpu - oracle| <= tol * magnitude``.  ReLU units whose FP64 pre-activation
lies within ``tol * magnitude`` of zero may legitimately switch either way in
float32; for them the oracle carries the midpoint of the two admissible
gradients and widens the magnitude to cover both.

Modules:
  field    -- level layout, hash/dense indexing, trilinear encoding, SH, MLP
  rays     -- camera rays, the FP32 position path, samplers, batch cut
  render   -- compositing (Eq. 5, 6), loss (Eq. 3, 4, 7) and their adjoints
  step     -- the whole mapping step and Adam
  covariance -- marginal covariances of the tracking Hessian (Eq. 1, 2)
"""
