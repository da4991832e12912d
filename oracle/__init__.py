"""FP64 CPU oracle for the improved MRT pseudopotential D2Q9 method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (``paper_1211_6932_amd``) and never imports it.

Modules:
  lbref  -- ctypes binding of lbref.c: the per-step update (Eqs. 1-7, 24, 25, 30)
  eos    -- Carnahan-Starling EOS, critical point, Maxwell rule, Eq. (21), Eq. (29)
  post   -- Laplace pressure jump, effective radius, interface width
  mlp    -- FP64 reference of the learned initialiser's network (forward/backward)
"""
