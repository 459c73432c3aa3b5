"""Plain FP64 CPU oracle for the TRSTMI candidate-coherence path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library (no kernels,
headers, helpers, constant tables or pre/post-processing) and it never
imports the ``paper_2207_06374_amd`` package.

Everything is written to be checked by eye against the paper
(Park, Saltijeral, Zhong, "Grassmannian packings: Trust-region stochastic
tuning for matrix incoherence", arXiv:2207.06374):

* ``coherence``  -- coherence of a frame (§I), Welch bound (§II),
  orthoplex / Levenshtein bounds (§V, Proposition on orthoplex and
  Levenshtein bounds), column normalisation (§IV, remark on dividing each
  column by its norm).
* ``miso``       -- the beamforming-codebook quantiser of §III (argmax of
  |<phi_i, h>|^2 over the codewords) and its Monte-Carlo distortion.
* ``philox``     -- Philox4x32-10 counter-based generator, from its published
  definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11).  The paper does not fix a generator; see ``rng``.
* ``rng``        -- the counter layout, uniforms and Box-Muller complex
  Gaussians used for the random start (Alg. 2 step 1) and the trust-region
  perturbations.
* ``rounding``   -- round-to-nearest-even to bfloat16 / float32, used to
  emulate the reduced-precision screening forms.
* ``smoothmax``  -- the shifted log-sum-exp smooth maximum of §IV over the
  upper-triangle Gram moduli (the objective the paper's optimiser uses).
* ``trust_region`` -- the trust-region step of the paper's optimiser:
  Steihaug CG (Alg. 1, read with the textbook's completion) on the smooth
  maximum, and the outer ratio test and radius update.
* ``trstmi``     -- Haar start, candidate generation, evaluation,
  select/accept and radius update, step and solve.

Every function is pinned in ``tests/test_oracle_*.py`` against something other
than itself (closed forms, brute force, known optimal frames, published
known-answer vectors, invariances, distributional tests).
"""

from .coherence import (  # noqa: F401
    normalize_columns,
    gram,
    coherence,
    coherence_sq_upper,
    coherence_pair,
    coherence_bruteforce,
    welch_bound,
    orthoplex_bound,
    levenshtein_bound,
    lower_bound,
)
from .miso import quantize, distortion  # noqa: F401
from .philox import philox4x32_10  # noqa: F401
from .rng import (  # noqa: F401
    TAG_PERTURB,
    TAG_HAAR,
    uniforms_from_words,
    box_muller,
    complex_gaussian_frame,
)
from .rounding import round_to_bf16, round_to_fp32  # noqa: F401
from .smoothmax import (  # noqa: F401
    upper_values,
    smooth_max_of_values,
    smooth_max,
    smooth_max_bruteforce,
    smooth_max_grad,
    smooth_max_hess_vec,
)
from .trust_region import (  # noqa: F401
    TRParams,
    TRReport,
    cg_steihaug,
    tr_step,
    rdot,
    OptParams,
    optimize,
)
from .trstmi import (  # noqa: F401
    Params,
    State,
    StepReport,
    haar_init,
    perturbations,
    make_candidates,
    evaluate_candidates,
    step,
    solve,
    screen_error_bound,
    split_screen_error_bound,
)
