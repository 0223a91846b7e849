"""Plain, slow, FP64 CPU oracle for the structure-preserving spectral division of
definite pseudosymmetric matrices (Benner, Nakatsukasa, Penke, arXiv 2203.08900).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_2203_08900_amd`` and its Python binding) imports, calls or links this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` do.  The oracle shares no code with the GPU path: it works on
the full 2m x 2m matrix H with the paper's own formulation (symmetric indefinite
LDL^T solves, Eq:LDLZolo), while the GPU path works on half-size SPD matrices.

Modules
-------
zolotarev   Zolotarev coefficients in multiprecision (Eq:Compcis, Eq:hatZ,
            Eq:ZPartialFrac, the l-recurrence of Alg. 8).
sign        Alg. 8 (hyperbolic Zolo-PD) taken literally with LDL^T solves on
            the full H, plus the plain-definition matrix sign function.
bases       Alg. 6 (Cholesky bases, with the sign of the Q_- formula corrected,
            see the module docstring), Alg. 7 (pivoted LDL^T bases) and Alg. 4.
divide      One step of Alg. 3 for definite H: bases, decoupled blocks
            (Thm. DefDivConq) and the paper's backward error.
eig         Plain-definition eigen-decomposition (simultaneous diagonalization
            of Sigma*H and Sigma, Thm. EVREalSigmaOrth), canonical ordering, and
            Alg. 2 (symmetric spectral divide-and-conquer) for the recursion.
grad        Daleckii-Krein reference gradient of trace(W P_+).
hermitian   The complex Bethe-Salpeter forms Eq:BSE1 and Eq:BSE2: sign(H) by the
            definite pencil and by the general eigensolver, Alg. 6 and H_+ in
            complex arithmetic.
"""
