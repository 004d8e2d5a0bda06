"""The mutation check of the oracle's pins (tests/oracle_mutations.py, run
directly) stays applicable: every mistake it plants replaces text that still
occurs in the oracle file it patches, and replaces it with something else."""
import os

import oracle_mutations as OM


def test_every_planted_mistake_still_matches_its_oracle_source():
    for group, (src_file, mutations, tests) in OM.GROUPS.items():
        src = open(os.path.join(OM.ORACLE, src_file)).read()
        for name, a, b in mutations:
            assert src.count(a) >= 1, (group, name)
            assert a != b, (group, name)
        for t in tests:
            assert os.path.exists(os.path.join(OM.HERE, t)), t
    assert OM.EXPECTED_SURVIVORS <= {n for _, m, _ in OM.GROUPS.values() for n, _, _ in m}
