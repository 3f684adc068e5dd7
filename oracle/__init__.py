"""CPU oracle of the nearest-neighbour certificate method: TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import anything under ``oracle/``.  The product path never does, and the
oracle never imports the product: the two share no code.

* ``model``    -- the state machine of the method (certificates, clock, filter,
                  repair, rebuild, entropy) in plain NumPy over a brute-force C
                  routine (``nncert_oracle.c``, built with gcc by ``model.build``);
* ``exact``    -- exact rational arithmetic for tiny inputs, used to pin the above;
* ``mlp``      -- the strategy selector's network in binary64 NumPy.
"""
