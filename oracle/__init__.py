"""FP64 CPU oracle of the JDE hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
imports, links or runs anything here, and this package imports nothing from
the product.  The only code both share is ``jde_inputs`` (seeded inputs).

Plain, slow and obviously correct: FP64 throughout (except the NMS overlap
predicate, which is evaluated in IEEE FP32 so that keep-indices are bit-exact,
see ``post.iou_exceeds``), with numpy's matmul/sort/linear solve and
scipy's linear_sum_assignment as the only library primitives.

Modules:
  network  -- direct convolution, leaky ReLU, residual, nearest x2 upsample,
              concat, the Darknet-53/FPN/heads forward (Sec. 3.1) and the
              batch-norm calibration used to make synthetic weights.
  post     -- anchor decode, confidence threshold, sort, greedy IoU NMS and
              embedding L2 normalisation (Appendix A, items 1-3).
  track    -- cosine cost with Mahalanobis gating, textbook Kalman filter,
              min-cost assignment and the track lifecycle (Appendix A, items 4-9).

Parity status: every function is pinned by tests/test_oracle_*.py against
brute force, closed forms or invariants; the network as a whole is pinned
only by composition of pinned layers (the paper prints no intermediate value).
"""
