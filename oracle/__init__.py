"""Oracle for the P-TRT lattice Boltzmann update (arXiv 2602.06686).

TEST INFRASTRUCTURE ONLY.  The modules here are the plain, slow, FP64 CPU
definitions that the GPU kernels are checked against:

* ``ptrt_oracle.c`` / ``ptrt.py`` -- the P-TRT update (Eq. PTRT) in plain C,
  collide then stream, with halfway bounce-back and a body force;
* ``trt_rlb.py`` -- the TRT-RLB update (Eq. TRT-RLB, Hermite projection and
  reconstruction, Eq. R2R3_hermite) written independently in NumPy; the
  paper's equivalence theorems say it gives the same post-collision state;
* ``analytic.py`` -- closed-form solutions used to pin both (Taylor-Green
  decay, Eq. TG; discrete Poiseuille profile under halfway bounce-back).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything here.  The product library
(``paper_2602_06686_amd``) never imports, links or calls the oracle, and the
oracle shares no code with it.
"""
