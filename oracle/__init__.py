"""Plain FP64 CPU oracle of the VOLDOR+ dense GEM hot path and keyframe alignment.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library; the two meet only through the
arrays the seeded input generator produces and through the window-parameter
dictionary (plain numbers).

Every function follows the paper (arXiv 2104.06800, "VOLDOR+SLAM") section or
equation it cites, and the readings of its silent or garbled points listed in
the design notes.  It is deliberately slow and direct: loops run over chain
positions and slots exactly as the method states them, vectorised only across
independent chains or pixels.

Modules
  philox   Philox4x32-10 counter-based draws (Salmon et al., SC'11)
  geometry rotations, pose update, reprojection, bilinear flow sampling
  fisk     log-logistic planar residual density, MIE energy terms, IRLS weight
  gem      E-step, M-step, pose step, depth priors, confidence, GEM iteration
  align    point-to-plane inverse-depth keyframe alignment
  vc       visibility-coverage scores for VO stride and keyframe selection
  pose_sample  Monte-Carlo P3P pose samples, meanshift mode and pose covariance
  proposal the learned depth / rigidness proposal network (forward, backward, Adam)
"""
from . import philox, geometry, fisk, gem, align, proposal, vc, pose_sample  # noqa: F401
