"""CPU FP64 oracle for the BOA Constrictor compressor -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy / Python-integer
implementation of what the compressor computes, written from the paper:

* ``model``  -- the byte-level Mamba predictor step (Models, Algorithm 1;
  Appendix A, discrete recurrence and selection mechanism), in float64.
* ``coder``  -- softmax, integer histogram / CDF and the range coder
  (Range coding: Probabilities and integer CDF, Encoder, Decoder).
* ``order2`` -- an adaptive order-2 context-count model driving the same
  coder (not in the paper; a fallback and a bits/byte yardstick).
* ``grad``   -- float64 reverse-mode gradients of the cross-entropy loss
  (Theoretical Framework, cross-entropy loss) and AdamW.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU library; its inputs come from ``synth``.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or library routines, except the
learned-gain comparison (``grad`` + training), which the paper gives no
synthetic-data numbers for ("parity unpinned" in absolute terms; only the
ordering trained < order-2 < untrained is tested).
"""
