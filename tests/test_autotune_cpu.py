"""CPU checks of the ragged-batch autotuner's bookkeeping: the team-size
ladder, the persisted table and the allocation rule (minimise the slowest
instance's predicted time within the compute units)."""
import json

import pytest

from paper_2408_05444_amd import autotune


def test_ladder_powers_of_two_to_eight_rows_per_work_group():
    assert autotune.ladder(1000, 256) == [1, 2, 4, 8, 16, 32, 64, 125]
    assert autotune.ladder(128, 256) == [1, 2, 4, 8, 16]
    assert autotune.ladder(5, 256) == [1]
    assert autotune.ladder(4096, 256) == [1, 2, 4, 8, 16, 32, 64, 128, 256]


def test_table_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    t = autotune.Table(path)
    assert t.get("k") is None
    t.put("k", {1: 10.0, 4: 3.5})
    t.save()
    t2 = autotune.Table(path)
    assert t2.get("k") == {1: 10.0, 4: 3.5}
    assert json.load(open(path)) == {"k": {"1": 10.0, "4": 3.5}}


def test_allocation_feeds_the_slowest_instance():
    # Instance 0: twice the work of instance 1; both scale perfectly.
    times = [{1: 40.0, 2: 20.0, 4: 10.0, 8: 5.0}, {1: 20.0, 2: 10.0, 4: 5.0, 8: 2.5}]
    teams = autotune.allocate(times, [100, 100], cus=10)
    # 8 + 2 = 10 work-groups; instance 0 at 5 us, instance 1 at 10 us would
    # be next to grow but only 0 work-groups remain.
    assert sum(teams) <= 10
    assert teams == [8, 2]
    # Weighting by updates reverses the order.
    teams = autotune.allocate(times, [10, 1000], cus=10)
    assert teams[1] > teams[0]


def test_allocation_stops_where_larger_teams_stop_helping():
    times = [{1: 30.0, 2: 20.0, 4: 21.0, 8: 25.0}]
    assert autotune.allocate(times, [1], cus=256) == [2]


def test_allocation_rejects_more_instances_than_units():
    with pytest.raises(ValueError):
        autotune.allocate([{1: 1.0}] * 3, [1, 1, 1], cus=2)
