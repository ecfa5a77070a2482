"""FP64 CPU oracle for the NNVISR frame-group enhancement path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of what the enhancement path computes, written from
the NNVISR paper (Tong, Hu, Wang, ACM MM 2023) and from the readings its
silences require.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  The device library never calls it, and it
shares no code with the device library; the two meet only through the seeded
arrays produced by ``synth``.

Modules
  pixel    -- Y'CbCr decode, chroma resampling, BT.709 matrices, padding, requantisation
  scene    -- integer scene-change metric, cut decision, frame grouping, frame-store layout
  network  -- conv3x3, LeakyReLU, modulated deformable conv (DCNv2), pixel shuffle, the
              extract / fusion stages of the generic enhancement network
  pipeline -- a frame group end to end, and a whole clip in stream order

Parity status: every function is pinned by the ``-m "not gpu"`` tests against
closed forms, published code values, brute force or library routines, except
the composed network as a whole, which is parity unpinned beyond the
composition of its pinned parts (there is no trained model or published
output to compare against).
"""
from . import pixel, scene, network, pipeline  # noqa: F401
