"""Oracle package — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU path
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import anything from here; the product package never
does, and nothing here imports the product package.

Contents
--------
``sweep``   naive FP64/FP32 Jacobi sweep of the four stencils (C, ``oracle.c``),
            the plain definition of the method's result (see ``sweep.py``).
``models``  the paper's cache-block-size and code-balance formulas.
``mlp``     FP64 forward/backward of the cost-model MLP (numpy).
"""
