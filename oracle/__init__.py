"""Reference oracle for the peridynamic MC/MLMC hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import, call or link anything here; the
product library never does.  The oracle is a plain, slow FP64 reading of the
method: unique-bond loops, the textbook stretch, no compensation, no fusion.

Modules:
  geometry  -- lattice, horizon neighbourhoods, notch cut, pads (NumPy)
  solver    -- problem assembly + ctypes binding of pd_oracle.c (time loop)
  kl        -- Karhunen-Loeve basis and lognormal field synthesis (NumPy)
  mlmc      -- MC / MLMC estimators and sample statistics (NumPy)
"""
