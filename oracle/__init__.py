"""Plain CPU oracle for the ByteStore scan / lookup path (arXiv 2209.00220).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  It shares no code with the HIP path (``paper_2209_00220_amd``) and
never imports it; the two meet only through the seeded input generator in
``datagen``.

Everything here is written for a reader to check against the paper by eye:
numpy slices stand in for the paper's loops, integers are exact (Python ints or
numpy unsigned types), and no step is blocked, fused or reordered.

Modules
-------
``dictionary``  sorted distinct values and their counts (Sec. 2.2, the
                order-preserving dictionary).
``ppe``         prefix-preserving encoding, numerical (Algorithm 1) and
                categorical (Algorithm 2).
``layout``      Bit-Packed (Sec. 2.3), ByteSlice (Sec. 2.5) and VBS (Sec. 3.2)
                in the paper's row order, plus decoders.
``scan``        the scan result bitvector (Sec. 2.2) on values, on padded codes,
                and the byte-serial early-stop classifier of Sec. 3.3 / Lemma 1.
``lookup``      lookup of values for row IDs or a result bitvector (Sec. 2.2),
                and Algorithm 4's bit-trick reconstruction.
``advisor``     profiling literals, area under the curve and the layout choice
                of Algorithm 5.

Readings of the paper where it is silent or inconsistent are listed in the
module docstrings and in the repository's design notes.
"""
