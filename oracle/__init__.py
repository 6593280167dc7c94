"""FP64 CPU oracle for the NLOS hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy/SciPy code, written from the paper
(López-Ruiz & Royo, "Memory-efficient GPU pipelines for real-time
non-line-of-sight reconstruction").  It shares no code with the HIP library in
``paper_2608_28183_amd/``; the two meet only at the seeded inputs of
``scenes/``.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path never
calls it and never falls back to it.

Modules
  dft      -- the DFT definition as a matrix product (exact index reduction)
  binning  -- photon-event histogramming (Section 4.1, photon binner)
  fk       -- f-k migration (Section 3.1 Eq. 1-2, Section 4.2, Algorithms 1-2)
  rsd      -- phasor DFT and radial RSD propagation (Section 4.3 Eq. 4-7,
              supplementary sampling rules, Algorithm 4) plus the exact dense
              and direct-sum RSD used as pins
  moe      -- mixture of experts of the two (Section 4.4, Eq. 10)
  merge    -- coherence-weighted temporal merging (Section 4.4, Eq. 8-9)
  metrics  -- error measures (relative L2, PSNR, argmax distance)

Every function states the passage it follows, and each module states the
readings it takes where the paper is silent or garbled.
"""
