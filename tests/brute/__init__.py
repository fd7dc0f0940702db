"""Pure-Python brute force of the whole estimator, for tiny fields.

A second CPU implementation, written independently of ``oracle/`` (it shares
no code with it and does not call it), that follows the same readings of the
paper: block sampling (Section 4.3), the ZFP side (Sections 4.2, 5.2) with
exact integer arithmetic and a literal group-testing coder, the SZ side
(Sections 4.1, 5.1) with the Lorenzo predictor and linear-scaling
quantization, the entropy of Eq. 5 with the Section 6.2 offset, and
Algorithm 1's selection.  The tests require it to agree with the C oracle bit
for bit.  Slow by design: tiny inputs only.
"""
