"""FP64 CPU oracle for the flow-based phi^4 sampler (arXiv 2208.08903).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only the tests, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; both sides take their inputs from ``seeded_inputs``.

Every function is a plain, slow, obviously correct restatement of what the paper
defines, in float64 NumPy, citing the passage it follows:

  prior    -- Gaussian prior r(z) (Sec. 1, prior distribution) and the
              Philox4x32-10 / Box-Muller draw used to realise it.
  action   -- lattice phi^4 action S (Sec. 1, action and potential equations)
              and its force dS/dphi.
  flow     -- checkerboard affine coupling layers with convolutional s/t nets
              (Sec. 1, coupling-layer and composition equations), log q, the
              shifted reverse-KL loss and its hand-derived adjoint gradient.
  mh       -- independence Metropolis-Hastings chain on log-weights (Sec. 1,
              the Metropolis-Hastings test "with the Jacobian").
  hmc      -- HMC baseline (Sec. 2.2, "HMC ... to compare results").
  adam     -- Adam update of the training loop (example parameter file).

Parity status of each function is recorded in its module header; every function
here is pinned by a test under ``tests/`` that checks it against closed forms,
invariants, brute force or published test vectors.
"""
