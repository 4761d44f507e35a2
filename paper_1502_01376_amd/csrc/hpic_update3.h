// hpic_update3.h -- work shape of the 3D k-space field update (solve.hip),
// shared with the host runtime that builds its work items.
#pragma once

namespace hp {

constexpr int KSTRIP3 = 8;  // planes i3 walked by one thread of the 3D update

}  // namespace hp
