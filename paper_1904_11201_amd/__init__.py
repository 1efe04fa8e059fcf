"""MI355X (gfx950) join library after "GPU-based Efficient Join Algorithms on Hadoop".

Submodules:
  join      -- Python binding of libjoin.so (include/join.h): hash_join, theta_join, join_count,
               join_materialize, join_hash, join_theta, join_scan_u64 over torch device tensors.
  datagen   -- seeded synthetic workloads (inputs only).
  build     -- compiles libjoin.so for gfx950 with hipcc.

The binding is imported explicitly (``from paper_1904_11201_amd import join``); it raises
ImportError when libjoin.so has not been built.
"""
