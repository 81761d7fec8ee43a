"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU reference for what the GPU SMMO library
computes (DynaSOAr, Springer & Masuhara, ECOOP 2019).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import anything from here.  It shares no code with the HIP path; the only
thing both start from is ``paper_1810_11765_amd.inputs`` (seeded starting
states, no method arithmetic).

Modules
  core.py      ctypes wrapper of oracle.c: RNG and the four workload simulators
  bitmap_ref   sequential hierarchical bitmap (Sec. 4.1, Alg. 3-5)
  block_ref    object-slot bitmap rules of a block (Alg. 6-9, App. A)
  layout_ref   block capacity and SOA layout (Sec. 3.2)
  heapcheck    invariant checker over a raw heap dump
"""
