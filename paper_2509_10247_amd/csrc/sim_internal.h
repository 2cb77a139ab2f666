// Definition of the opaque sim_handle shared by the host-side translation units.
#pragma once

#include <vector>

#include "kernels.h"

struct SensorBuf {
  da::SensorDev dev;
  void* mem = nullptr;
};

struct sim_handle {
  sim_config cfg{};
  SensorBuf cam, lidar;
  da::SceneDev scene;
  int32_t* agent_env = nullptr;        // owned [A]
  int32_t* agent_off_owned = nullptr;  // owned [E+1] when the caller passes NULL
  const float* params = nullptr;       // SoA [P][A]: params_owned once set
  float* params_owned = nullptr;       // owned copy of the caller's parameters
  std::vector<int32_t> host_sph_off, host_box_off, host_cyl_off, host_agent_off;
  int n_sph = 0, n_box = 0, n_cyl = 0;
  bool has_scene = false;
  void* rollout = nullptr;             // uneven-batch rollout plan (rollout.hip)
  int render_nt = 256;                 // threads per agent of the launch-per-op render (128 or 256)
};

void rollout_plan_free(sim_handle* h);

// the simulator and configuration a BPTT handle was created with
sim_handle* bptt_sim_of(const bptt_handle* b);
const bptt_config* bptt_cfg_of(const bptt_handle* b);
