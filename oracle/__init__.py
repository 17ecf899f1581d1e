"""CPU oracle for the RapidPT hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy/SciPy implementation of what the permutation-testing
path computes, written from the paper (Gutierrez-Barragan et al., "Accelerating
Permutation Testing in Voxel-wise Analysis through Subspace Tracking"):

* ``tstat``      -- the two-sample t statistic (Sec. 3.2, Eq. 2) and NaivePT
                    (Sec. 2.1, Alg. 1);
* ``philox``     -- the counter-based Philox4x32-10 generator (Salmon et al.,
                    SC'11) and the Box-Muller transform, used for the residual
                    noise draw of Alg. 2;
* ``rapidpt``    -- RapidPT training and recovery (Sec. 4, Alg. 2);
* ``sampling``   -- relabellings, sampled sets and the start basis drawn from
                    a seed (Philox words driving a partial Fisher-Yates
                    shuffle; Alg. 1, Alg. 2);
* ``masked_loss``-- the masked completion loss of Eq. 1 and its gradient;
* ``metrics``    -- KL divergence, thresholds, p-values and the resampling
                    risk of Sec. 5.5 (Eq. 4).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1703_01506_amd``) and never imports it; the only common code is the
seeded input generator package ``rpt_synth``, which holds none of the
method's arithmetic.

Parity status per function is listed in each module's header.  Every function
here is pinned by a ``-m "not gpu"`` test against something other than itself
(hand values, brute force, closed forms, invariants, published test vectors)
except where a header says "parity unpinned".
"""

